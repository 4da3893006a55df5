// Discrete adjoint of the fluctuating two-species D2Q9 step (FP64 storage,
// one replica), with the noise stream held fixed.
//
// Forward step t (see k_step.hip): f(t) = pull(S_t) (streaming with mid-way
// bounce-back), densities rho^S, the non-ideal force of Eq. (11) with the a_*
// correction of the footnote to Eq. (13) and the non-equilibrium force of
// Eq. (12), the wall U_z fix of Sec. III.A, the barycentric velocity of
// Eq. (10), and the moment-space collision of Eqs. (14)-(15) with forcing
// moments and the noise of Eqs. (22)-(23); S_{t+1}(r) = post-collision
// populations of r (plus constant row shifts).
//
// With mu_{t+1} = dJ/dS_{t+1}, one adjoint step computes mu_t = dJ/dS_t and
// the parameter sensitivities:
//  1. k_adj_density: full densities of f(t) (the non-local force reads them).
//  2. k_adj_local: per node, the forward collision is recomputed and reversed:
//     adjoints of the node's 18 pre-collision populations (local
//     dependencies, including the node's own densities and, on sample steps,
//     the structure-factor term), adjoints of the force stencil sums s^A, s^B,
//     and the node's share of dJ/d(lambda_s, lambda_d, G).
//  3. k_adj_gather: every node collects the stencil adjoints of the nodes
//     whose force reads its densities (ghost rows fold onto the wall row) and
//     pushes the adjoint of each pre-collision population back to the stored
//     element it was pulled from.
//  4. k_adj_theta, once after the reverse sweep: fixed-order (strided, then
//     tree) sum of the per-block parameter partials, which each block of
//     k_adj_local (and of k_adj_psample) adds to over the steps in order.
// The structure-factor term of a sample step is dJ/d dphi(r) =
// (Lx Lz)^{-1/2} Re sum_{q in half spectrum} G(q) e^{+i q.r} with
// G(q) = (2 w_q (S(q) - S*(q))) * 2 (Phi(q) - <Phi(q)>) / n, evaluated with
// direct sums (k_adj_rows_fwd, k_adj_cols_fwd, k_adj_cols_inv, k_adj_rows_inv).
#include "fnlb.h"
#include "fnlb_device.hpp"
#include "fnlb_fft.hpp"
#include "fnlb_internal.hpp"
#include "fnlb_state.hpp"

namespace fnlb {
namespace {

constexpr int kCXa[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kCZa[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr double kWa[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                           1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
// basis of Table I, T[a][l], and N_a
constexpr double kT[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {-2, 1, 1, 1, 1, 4, 4, 4, 4},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, -1, 0, 1, 0, 2, -2, -2, 2},
    {0, 0, -1, 0, 1, 2, 2, -2, -2},
    {2, -4, -4, -4, -4, 8, 8, 8, 8}};
constexpr double kN[9] = {1.0, 1.0 / 3, 1.0 / 3, 4.0, 4.0 / 9, 1.0 / 9, 2.0 / 3, 2.0 / 3, 16.0};

struct AdjArgs {
  const RepInfo* rep;      // the replica (device)
  const double* state;     // S_t (deviations, FP64)
  const double* mu_next;   // dJ/dS_{t+1}
  double* mu;              // dJ/dS_t (output)
  double* dens;            // [2][Lz][Lx] full densities of f(t)
  double* gf;              // [18][Lz][Lx] local adjoints of the pulled populations
  double* gs;              // [4][Lz][Lx] adjoints of s^A_x, s^A_z, s^B_x, s^B_z
  const double* adjfield;  // [Lz][Lx] dJ/d dphi of this sample, or null
  int32_t field;           // 0: delta c, 1: delta rho
  int64_t t;               // time of the step (keys the noise)
  double* tpart;           // [blocks][3] partial dJ/d(lambda_s, lambda_d, G)
};

__global__ void k_adj_density(const AdjArgs a) {
  const RepInfo& R = *a.rep;
  const int Lx = R.Lx, Lz = R.Lz;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= Lx * Lz) return;
  const int j = n / Lx, x = n - j * Lx;
  const uint32_t link_b = 64u * 8u, row_b = (uint32_t)R.pitch * 18u * 8u;
  const Rsrc in = make_rsrc(a.state, (uint32_t)(18 * R.plane * 8));
  const int xm = x == 0 ? Lx - 1 : x - 1, xp = x == Lx - 1 ? 0 : x + 1;
  double o[18];
  load_pulled(in, link_b, row_b, j, Lz, col_offset(x, 8), col_offset(xm, 8), col_offset(xp, 8),
              o);
  double da = 0, db = 0;
  for (int l = 0; l < 9; ++l) {
    da += o[l];
    db += o[9 + l];
  }
  const double rA = R.rA_mid + R.rA_step * j;
  a.dens[n] = rA + da;
  a.dens[Lx * Lz + n] = (R.rho0 - rA) + db;
}

// Three block sums at once, each added in the order block_sum adds it (the
// same butterfly, then the wavefront totals in wavefront order), behind one
// pair of barriers.  sh holds 3 doubles per wavefront.
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* sh) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    a += __shfl_xor(a, m, 64);
    b += __shfl_xor(b, m, 64);
    c += __shfl_xor(c, m, 64);
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sh[3 * w] = a;
    sh[3 * w + 1] = b;
    sh[3 * w + 2] = c;
  }
  __syncthreads();
  double sa = 0, sb = 0, sc = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
    sa += sh[3 * k];
    sb += sh[3 * k + 1];
    sc += sh[3 * k + 2];
  }
  a = sa;
  b = sb;
  c = sc;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
  return s;
}

__global__ __launch_bounds__(256) void k_adj_local(const AdjArgs a) {
  __shared__ double sh[12];  // 3 per wavefront
  const RepInfo& R = *a.rep;
  const int Lx = R.Lx, Lz = R.Lz, N = Lx * Lz;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double th_s = 0, th_d = 0, th_g = 0;
  if (n < N) {
    const int j = n / Lx, x = n - j * Lx;
    const bool bot = j == 0, top = j == Lz - 1;
    const uint32_t link_b = 64u * 8u, row_b = (uint32_t)R.pitch * 18u * 8u;
    const Rsrc in = make_rsrc(a.state, (uint32_t)(18 * R.plane * 8));
    const int xm = x == 0 ? Lx - 1 : x - 1, xp = x == Lx - 1 ? 0 : x + 1;
    double f[2][9];
    {
      double o[18];
      load_pulled(in, link_b, row_b, j, Lz, col_offset(x, 8), col_offset(xm, 8),
                  col_offset(xp, 8), o);
      for (int l = 0; l < 9; ++l) {
        f[0][l] = o[l];
        f[1][l] = o[9 + l];
      }
    }
    const double* dA = a.dens;
    const double* dB = a.dens + N;
    const double rS[2] = {dA[n], dB[n]};
    const double rho = rS[0] + rS[1];
    // stencil sums s^S = sum_{m>=1} w_m c_m rho^S(r + c_m), ghost rows = wall row
    double s[2][2] = {{0, 0}, {0, 0}};
    for (int m = 1; m < 9; ++m) {
      int xx = x + kCXa[m];
      xx = xx < 0 ? xx + Lx : (xx >= Lx ? xx - Lx : xx);
      int jj = j + kCZa[m];
      jj = jj < 0 ? 0 : (jj > Lz - 1 ? Lz - 1 : jj);
      const int k = jj * Lx + xx;
      s[0][0] += kWa[m] * kCXa[m] * dA[k];
      s[0][1] += kWa[m] * kCZa[m] * dA[k];
      s[1][0] += kWa[m] * kCXa[m] * dB[k];
      s[1][1] += kWa[m] * kCZa[m] * dB[k];
    }
    const double G = R.G, ne = R.ne_coef;
    // forces: a_bar = -G (rho^A s^B + rho^B s^A) / rho
    double Q[2], ab[2], F[2][2];
    for (int d = 0; d < 2; ++d) {
      Q[d] = rS[0] * s[1][d] + rS[1] * s[0][d];
      ab[d] = -G * Q[d] / rho;
      F[0][d] = rS[0] * ab[d];
      F[1][d] = rS[1] * ab[d];
    }
    F[0][1] += ne * rho;
    F[1][1] -= ne * rho;
    // pre-fix momenta
    double jx[2], jz[2];
    for (int sp = 0; sp < 2; ++sp) {
      jx[sp] = 0;
      jz[sp] = 0;
      for (int l = 0; l < 9; ++l) {
        jx[sp] += kCXa[l] * f[sp][l];
        jz[sp] += kCZa[l] * f[sp][l];
      }
    }
    // wall fix
    double ft[2][9];
    for (int sp = 0; sp < 2; ++sp)
      for (int l = 0; l < 9; ++l) ft[sp][l] = f[sp][l];
    const bool wall = bot || top;
    double Pi = 0, del[2] = {0, 0};
    if (wall) {
      Pi = jz[0] + jz[1] + 0.5 * (F[0][1] + F[1][1]);
      for (int sp = 0; sp < 2; ++sp) {
        del[sp] = rS[sp] / rho * Pi;
        if (bot) {
          ft[sp][2] -= del[sp];
          ft[sp][0] += del[sp];
        } else {
          ft[sp][4] += del[sp];
          ft[sp][0] -= del[sp];
        }
      }
    }
    double jtx[2], jtz[2];
    for (int sp = 0; sp < 2; ++sp) {
      jtx[sp] = jx[sp];
      jtz[sp] = jz[sp] - del[sp];
    }
    const double Ux = (jtx[0] + jtx[1] + 0.5 * (F[0][0] + F[1][0])) / rho;
    const double Uz = (jtz[0] + jtz[1] + 0.5 * (F[0][1] + F[1][1])) / rho;

    // noise: the same 14 normals as the forward step
    const uint32_t node = (uint32_t)(j * Lx + x);
    double g[16];
    // one call at a time (not unrolled): the table-driven FP64 Box-Muller of
    // three calls interleaved would raise the register pressure of this kernel
#pragma unroll 1
    for (uint32_t call = 0; call < 3; ++call) {
      double q4[4];
      node_normals(node, (uint64_t)a.t, call, R.seed_lo, R.seed_hi, q4, R.bm);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (c == (int)call) g[4 * c + i] = q4[i];
    }
    {
      // g_12, g_13: this step's half of the call shared with the other step
      // of its pair
      uint32_t w12, w13, o12, o13;
      shared_words(node, (uint64_t)a.t, R.seed_lo, R.seed_hi, w12, w13, o12, o13);
      box_muller(w12, w13, g[12], g[13], R.bm);
      g[14] = g[15] = 0.0;
    }
    // gaussian index of moment a for species A / B (a = 3..8); a = 1,2 use g0, g1
    const int gA[9] = {0, 0, 1, 2, 3, 4, 5, 6, 7};
    const int gB[9] = {0, 0, 1, 8, 9, 10, 11, 12, 13};
    const double lam[9] = {0, R.lam[1], R.lam[2], R.lam[3], R.lam[4],
                           R.lam[5], R.lam[6], R.lam[7], R.lam[8]};
    const double lam_s = R.lam[4], lam_d = R.lam[1];

    // ---- reverse pass ----
    double gft[2][9], gU[2] = {0, 0}, gF[2][2] = {{0, 0}, {0, 0}}, grS[2] = {0, 0};
    for (int sp = 0; sp < 2; ++sp) {
      double mus[9];
      for (int l = 0; l < 9; ++l) mus[l] = a.mu_next[state_index(9 * sp + l, j, x, R.pitch)];
      // forward moments of this species (post-fix)
      double m[9];
      for (int aa = 0; aa < 9; ++aa) {
        m[aa] = 0;
        for (int l = 0; l < 9; ++l) m[aa] += kT[aa][l] * ft[sp][l];
      }
      const double rs = rS[sp], Fx = F[sp][0], Fz = F[sp][1];
      const double meq[9] = {0, rs * Ux, rs * Uz, 3 * rs * (Ux * Ux + Uz * Uz),
                             rs * (Ux * Ux - Uz * Uz), rs * Ux * Uz, 0, 0, 0};
      const double Sm[9] = {0, Fx, Fz, 6 * (Ux * Fx + Uz * Fz), 2 * (Ux * Fx - Uz * Fz),
                            Ux * Fz + Uz * Fx, 0, 0, 0};
      // adjoint moments M_a = sum_l w_l T_al mu*_l / N_a
      double M[9];
      for (int aa = 0; aa < 9; ++aa) {
        M[aa] = 0;
        for (int l = 0; l < 9; ++l) M[aa] += kWa[l] * kT[aa][l] * mus[l];
        M[aa] /= kN[aa];
      }
      // f* = ft + R: direct path
      for (int l = 0; l < 9; ++l) gft[sp][l] = mus[l];
      double gm[9], gmeq[9], gS[9];
      for (int aa = 1; aa < 9; ++aa) {
        gm[aa] = -lam[aa] * M[aa];
        gmeq[aa] = lam[aa] * M[aa];
        gS[aa] = R.fac[aa] * M[aa];
      }
      // parameter sensitivities (relaxation, forcing factor, noise amplitude)
      for (int aa = 1; aa < 9; ++aa) {
        if (aa != 1 && aa != 2 && aa != 4 && aa != 5) continue;
        const double ll = lam[aa];
        double sig, gi, sign = 1.0;
        if (aa <= 2) {
          sig = R.sig[0][1];
          gi = g[aa - 1];
          if (sp == 1) sign = -1.0;  // xi^B_{1,2} = -xi^A_{1,2}
        } else {
          sig = R.sig[sp][aa];
          gi = g[sp == 0 ? gA[aa] : gB[aa]];
        }
        // d sigma / d lambda from sigma^2 = c lambda (2 - lambda)
        const double dsig = sig > 0 ? sig * (1.0 - ll) / (ll * (2.0 - ll)) : 0.0;
        const double d = (meq[aa] - m[aa]) * M[aa] - 0.5 * Sm[aa] * M[aa] +
                         sign * dsig * gi * M[aa];
        if (aa <= 2)
          th_d += d;
        else
          th_s += d;
      }
      (void)lam_s;
      (void)lam_d;
      // moments -> populations
      for (int l = 0; l < 9; ++l) {
        double acc = 0;
        for (int aa = 1; aa < 9; ++aa) acc += kT[aa][l] * gm[aa];
        gft[sp][l] += acc;
      }
      // m^eq(rho^S, U)
      grS[sp] += Ux * gmeq[1] + Uz * gmeq[2] + 3 * (Ux * Ux + Uz * Uz) * gmeq[3] +
                 (Ux * Ux - Uz * Uz) * gmeq[4] + Ux * Uz * gmeq[5];
      gU[0] += rs * (gmeq[1] + 6 * Ux * gmeq[3] + 2 * Ux * gmeq[4] + Uz * gmeq[5]);
      gU[1] += rs * (gmeq[2] + 6 * Uz * gmeq[3] - 2 * Uz * gmeq[4] + Ux * gmeq[5]);
      // forcing source moments S(U, F^S)
      gF[sp][0] += gS[1] + 6 * Ux * gS[3] + 2 * Ux * gS[4] + Uz * gS[5];
      gF[sp][1] += gS[2] + 6 * Uz * gS[3] - 2 * Uz * gS[4] + Ux * gS[5];
      gU[0] += 6 * Fx * gS[3] + 2 * Fx * gS[4] + Fz * gS[5];
      gU[1] += 6 * Fz * gS[3] - 2 * Fz * gS[4] + Fx * gS[5];
    }
    // U = (jt^A + jt^B + (F^A + F^B)/2) / rho
    double grho = -(Ux * gU[0] + Uz * gU[1]) / rho;
    for (int sp = 0; sp < 2; ++sp) {
      for (int l = 0; l < 9; ++l) gft[sp][l] += (kCXa[l] * gU[0] + kCZa[l] * gU[1]) / rho;
      gF[sp][0] += 0.5 * gU[0] / rho;
      gF[sp][1] += 0.5 * gU[1] / rho;
    }
    // wall fix: ft = f except the moved delta; jt_z is the moment of ft
    double gfp[2][9];
    for (int sp = 0; sp < 2; ++sp)
      for (int l = 0; l < 9; ++l) gfp[sp][l] = gft[sp][l];
    if (wall) {
      double gPi = 0;
      for (int sp = 0; sp < 2; ++sp) {
        const double gdel = bot ? (gft[sp][0] - gft[sp][2]) : (gft[sp][4] - gft[sp][0]);
        gPi += rS[sp] / rho * gdel;
        grS[sp] += Pi / rho * gdel;
        grho -= rS[sp] * Pi / (rho * rho) * gdel;
      }
      for (int sp = 0; sp < 2; ++sp) {
        for (int l = 0; l < 9; ++l) gfp[sp][l] += kCZa[l] * gPi;
        gF[sp][1] += 0.5 * gPi;
      }
    }
    // forces
    double gab[2];
    for (int d = 0; d < 2; ++d) {
      gab[d] = rS[0] * gF[0][d] + rS[1] * gF[1][d];
      grS[0] += ab[d] * gF[0][d];
      grS[1] += ab[d] * gF[1][d];
    }
    grho += ne * (gF[0][1] - gF[1][1]);
    double gQ[2];
    for (int d = 0; d < 2; ++d) {
      gQ[d] = -G * gab[d] / rho;
      th_g += -Q[d] * gab[d] / rho;
      grho += -ab[d] * gab[d] / rho;
    }
    double gs_out[2][2];
    for (int d = 0; d < 2; ++d) {
      grS[0] += s[1][d] * gQ[d];
      grS[1] += s[0][d] * gQ[d];
      gs_out[1][d] = rS[0] * gQ[d];  // s^B
      gs_out[0][d] = rS[1] * gQ[d];  // s^A
    }
    grS[0] += grho;
    grS[1] += grho;
    // sample term: the pressure's density adjoints, or a structure factor's
    if (a.adjfield && a.field == kAdjPressure) {
      grS[0] += a.adjfield[n];
      grS[1] += a.adjfield[(size_t)N + n];
    } else if (a.adjfield) {
      const double v = a.adjfield[n];
      if (a.field == 0) {  // delta c = rho^A / rho - c_0
        grS[0] += v * rS[1] / (rho * rho);
        grS[1] -= v * rS[0] / (rho * rho);
      } else {
        grS[0] += v;
        grS[1] += v;
      }
    }
    for (int sp = 0; sp < 2; ++sp)
      for (int l = 0; l < 9; ++l) a.gf[(size_t)(9 * sp + l) * N + n] = gfp[sp][l] + grS[sp];
    a.gs[0 * (size_t)N + n] = gs_out[0][0];
    a.gs[1 * (size_t)N + n] = gs_out[0][1];
    a.gs[2 * (size_t)N + n] = gs_out[1][0];
    a.gs[3 * (size_t)N + n] = gs_out[1][1];
  }
  block_sum3(th_s, th_d, th_g, sh);
  if (threadIdx.x == 0) {  // running partials of this block over the reverse sweep
    a.tpart[3 * blockIdx.x + 0] += th_s;
    a.tpart[3 * blockIdx.x + 1] += th_d;
    a.tpart[3 * blockIdx.x + 2] += th_g;
  }
}

// Node r collects the stencil adjoints of the nodes whose force reads its
// densities, then each pulled population's adjoint goes back to the stored
// element it came from (a permutation: no two nodes write one element).
__global__ void k_adj_gather(const AdjArgs a) {
  const RepInfo& R = *a.rep;
  const int Lx = R.Lx, Lz = R.Lz, N = Lx * Lz;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const int j = r / Lx, x = r - j * Lx;
  // the stencil adjoints of the eight nodes that read this one, all requested
  // before any is used (a row beyond a wall reads this node's row instead,
  // and its term is skipped below)
  double g[8][4];
#pragma unroll
  for (int m = 1; m < 9; ++m) {
    const int cx = kCXa[m], cz = kCZa[m];
    int xn = x - cx;
    xn = xn < 0 ? xn + Lx : (xn >= Lx ? xn - Lx : xn);
    const int jn = j - cz;
    const int k = (jn >= 0 && jn < Lz ? jn : j) * Lx + xn;
#pragma unroll
    for (int c = 0; c < 4; ++c) g[m - 1][c] = a.gs[c * (size_t)N + k];
  }
  double D[2] = {0, 0};
#pragma unroll
  for (int m = 1; m < 9; ++m) {
    const int cx = kCXa[m], cz = kCZa[m];
    int xn = x - cx;
    xn = xn < 0 ? xn + Lx : (xn >= Lx ? xn - Lx : xn);
    // regular: node (x - c_x, j - c_z) reads this node through link m
    const int jn = j - cz;
    if (jn >= 0 && jn < Lz) {
      for (int sp = 0; sp < 2; ++sp)
        D[sp] += kWa[m] * (cx * g[m - 1][2 * sp] + cz * g[m - 1][2 * sp + 1]);
    }
    // ghost: a wall-row node whose link m leaves the fluid reads the wall row
    if ((j == 0 && cz == -1) || (j == Lz - 1 && cz == 1)) {
      const int k = j * Lx + xn;
      for (int sp = 0; sp < 2; ++sp)
        D[sp] += kWa[m] * (cx * a.gs[(2 * sp) * (size_t)N + k] +
                           cz * a.gs[(2 * sp + 1) * (size_t)N + k]);
    }
  }
  const int pitch = R.pitch;
  const int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  for (int sp = 0; sp < 2; ++sp)
    for (int l = 0; l < 9; ++l) {
      const double v = a.gf[(size_t)(9 * sp + l) * N + r] + D[sp];
      // stored source of f_l(x, j): (x - c_lx, j - c_lz), or link opp(l) of
      // this node where that lies beyond a wall
      const int js = j - kCZa[l];
      size_t e;
      if (js < 0 || js >= Lz) {
        e = state_index(9 * sp + opp[l], j, x, pitch);
      } else {
        int xs = x - kCXa[l];
        xs = xs < 0 ? xs + Lx : (xs >= Lx ? xs - Lx : xs);
        e = state_index(9 * sp + l, js, xs, pitch);
      }
      a.mu[e] = v;
    }
}

// One block of 256 threads: strided partial sums in a fixed order, then a
// fixed-shape tree; the same result on every run for a given block count.
__global__ void k_adj_theta(const double* tpart, int nblocks, double* acc) {
  __shared__ double sh[3][256];
  const int t = threadIdx.x;
  double s0 = 0, s1 = 0, s2 = 0;
  for (int b = t; b < nblocks; b += 256) {
    s0 += tpart[3 * b];
    s1 += tpart[3 * b + 1];
    s2 += tpart[3 * b + 2];
  }
  sh[0][t] = s0;
  sh[1][t] = s1;
  sh[2][t] = s2;
  for (int h = 128; h >= 1; h >>= 1) {
    __syncthreads();
    if (t < h) {
      sh[0][t] += sh[0][t + h];
      sh[1][t] += sh[1][t + h];
      sh[2][t] += sh[2][t + h];
    }
  }
  if (t == 0) {
    acc[0] += sh[0][0];
    acc[1] += sh[1][0];
    acc[2] += sh[2][0];
  }
}

// ---- structure-factor misfit and its spectral adjoint (direct sums) ----

struct SpecArgs {
  const RepInfo* rep;
  const double2* tw;      // e^{-2 pi i m / Lx} (Lx entries) then e^{-2 pi i m / Lz}
  const double* acc;      // forward sums [2][3][nkx][Lz] of the replica (column-major)
  const double* target;   // S* [Lz][nkx]
  const double* weight;   // w  [Lz][nkx]
  double* Wq;             // 2 w (S - S*)          [Lz][nkx]
  double2* mean;          // <Phi>                 [Lz][nkx]
  double* Jpart;          // per-block partial J
  int32_t field;
  double nsamp;
  const double* dens;     // [2][Lz][Lx] full densities of the sampled state
  double2* rows;          // [Lz][nkx] row transforms / inverse column sums
  double2* Gq;            // [Lz][nkx]
  double* adjfield;       // [Lz][Lx]
};

__global__ void k_adj_misfit(const SpecArgs a) {
  __shared__ double sh[4];
  const RepInfo& R = *a.rep;
  const int nkx = R.Lx / 2 + 1, P = R.Lz * nkx;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  double part = 0;
  if (q < P) {
    const size_t plane = (size_t)P;
    const double* a2 = a.acc + (size_t)a.field * 3 * plane;
    const double n = a.nsamp;
    const int kz = q / nkx, kx = q - kz * nkx;
    const size_t qa = (size_t)kx * R.Lz + kz;  // the accumulators are [k_x][k_z]
    const double mr = a2[plane + qa] / n, mi = a2[2 * plane + qa] / n;
    const double S = a2[qa] / n - (mr * mr + mi * mi);
    const double d = S - a.target[q];
    a.Wq[q] = 2.0 * a.weight[q] * d;
    a.mean[q] = make_double2(mr, mi);
    part = a.weight[q] * d * d;
  }
  const double b = block_sum(part, sh);
  if (threadIdx.x == 0) a.Jpart[blockIdx.x] = b;
}

__device__ __forceinline__ double sample_field(const SpecArgs& a, const RepInfo& R, int j, int x) {
  const int N = R.Lx * R.Lz;
  const double rA = a.dens[j * R.Lx + x], rB = a.dens[N + j * R.Lx + x];
  if (a.field == 0) return rA / (rA + rB) - (R.rA_mid + R.rA_step * j) / R.rho0;
  return rA + rB - R.rho0;
}

// rows[j][kx] = sum_x dphi(x, j) e^{-2 pi i kx x / Lx}
__global__ void k_adj_rows_fwd(const SpecArgs a) {
  const RepInfo& R = *a.rep;
  const int Lx = R.Lx, nkx = Lx / 2 + 1;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= R.Lz * nkx) return;
  const int j = q / nkx, kx = q - j * nkx;
  double re = 0, im = 0;
  int m = 0;
  for (int x = 0; x < Lx; ++x) {
    const double v = sample_field(a, R, j, x);
    const double2 w = a.tw[m];
    re += v * w.x;
    im += v * w.y;
    m += kx;
    if (m >= Lx) m -= Lx;
  }
  a.rows[q] = make_double2(re, im);
}

// Phi(kz, kx) = (Lx Lz)^{-1/2} sum_j rows[j][kx] e^{-2 pi i kz j / Lz};
// G = W (2 / n) (Phi - <Phi>)
__global__ void k_adj_cols_fwd(const SpecArgs a) {
  const RepInfo& R = *a.rep;
  const int Lz = R.Lz, nkx = R.Lx / 2 + 1;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Lz * nkx) return;
  const int kz = q / nkx, kx = q - kz * nkx;
  const double2* twz = a.tw + R.Lx;
  double re = 0, im = 0;
  int m = 0;
  for (int j = 0; j < Lz; ++j) {
    const double2 v = a.rows[j * nkx + kx], w = twz[m];
    re += v.x * w.x - v.y * w.y;
    im += v.x * w.y + v.y * w.x;
    m += kz;
    if (m >= Lz) m -= Lz;
  }
  re *= R.inv_norm;
  im *= R.inv_norm;
  const double c = a.Wq[q] * 2.0 / a.nsamp;
  a.Gq[q] = make_double2(c * (re - a.mean[q].x), c * (im - a.mean[q].y));
}

// rows[j][kx] = sum_kz G(kz, kx) e^{+2 pi i kz j / Lz}
__global__ void k_adj_cols_inv(const SpecArgs a) {
  const RepInfo& R = *a.rep;
  const int Lz = R.Lz, nkx = R.Lx / 2 + 1;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Lz * nkx) return;
  const int j = q / nkx, kx = q - j * nkx;
  const double2* twz = a.tw + R.Lx;
  double re = 0, im = 0;
  int m = 0;
  for (int kz = 0; kz < Lz; ++kz) {
    const double2 v = a.Gq[kz * nkx + kx], w = twz[m];  // conj(w) = e^{+i...}
    re += v.x * w.x + v.y * w.y;
    im += v.y * w.x - v.x * w.y;
    m += j;
    if (m >= Lz) m -= Lz;
  }
  a.rows[q] = make_double2(re, im);
}

// adjfield(x, j) = (Lx Lz)^{-1/2} Re sum_{kx=0}^{Lx/2} rows[j][kx] e^{+2 pi i kx x / Lx}
__global__ void k_adj_rows_inv(const SpecArgs a) {
  const RepInfo& R = *a.rep;
  const int Lx = R.Lx, nkx = Lx / 2 + 1;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= Lx * R.Lz) return;
  const int j = n / Lx, x = n - j * Lx;
  double re = 0;
  int m = 0;
  for (int kx = 0; kx < nkx; ++kx) {
    const double2 v = a.rows[j * nkx + kx], w = a.tw[m];
    re += v.x * w.x + v.y * w.y;  // Re(v conj(w))
    m += x;
    if (m >= Lx) m -= Lx;
  }
  a.adjfield[n] = re * R.inv_norm;
}

// ---- the same four transforms by in-LDS FFTs (power-of-two lattices) ----

// one block per row j: rows[j][kx], kx = 0..Lx/2
__global__ void k_adj_rows_fwd_fft(const SpecArgs a) {
  extern __shared__ double2 lds[];
  const RepInfo& R = *a.rep;
  const int Lx = R.Lx, nkx = Lx / 2 + 1, bits = __ffs(Lx) - 1, j = blockIdx.x;
  double2* tws = lds + Lx;
  for (int x = threadIdx.x; x < Lx; x += blockDim.x)
    lds[bitrev(x, bits)] = make_double2(sample_field(a, R, j, x), 0.0);
  for (int m = threadIdx.x; m < Lx / 2; m += blockDim.x) tws[m] = a.tw[m];
  lds_fft(lds, bits, 1, tws);
  for (int k = threadIdx.x; k < nkx; k += blockDim.x) a.rows[(size_t)j * nkx + k] = lds[k];
}

// one block per tile of 2^lt columns: Phi = norm FFT_z(rows), then G
__global__ void k_adj_cols_fwd_fft(const SpecArgs a, int lt) {
  extern __shared__ double2 lds[];
  const RepInfo& R = *a.rep;
  const int M = R.Lz, nkx = R.Lx / 2 + 1, bits = __ffs(M) - 1, T = 1 << lt;
  const int kx0 = blockIdx.x << lt, nc = min(T, nkx - kx0), total = M << lt;
  double2* tws = lds + total;
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int j = q >> lt, c = q & (T - 1);
    if (c < nc) lds[c * M + bitrev(j, bits)] = a.rows[(size_t)j * nkx + kx0 + c];
  }
  for (int m = threadIdx.x; m < M / 2; m += blockDim.x) tws[m] = a.tw[R.Lx + m];
  lds_fft(lds, bits, nc, tws);
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int c = q >> bits, kz = q & (M - 1);
    if (c >= nc) continue;
    const double2 P = lds[c * M + kz];
    const size_t o = (size_t)kz * nkx + kx0 + c;
    const double cw = a.Wq[o] * 2.0 / a.nsamp;
    a.Gq[o] = make_double2(cw * (P.x * R.inv_norm - a.mean[o].x),
                           cw * (P.y * R.inv_norm - a.mean[o].y));
  }
}

// one block per tile of columns: rows[j][kx] = sum_kz G e^{+2 pi i kz j / Lz},
// as the conjugate of the forward FFT of conj(G)
__global__ void k_adj_cols_inv_fft(const SpecArgs a, int lt) {
  extern __shared__ double2 lds[];
  const RepInfo& R = *a.rep;
  const int M = R.Lz, nkx = R.Lx / 2 + 1, bits = __ffs(M) - 1, T = 1 << lt;
  const int kx0 = blockIdx.x << lt, nc = min(T, nkx - kx0), total = M << lt;
  double2* tws = lds + total;
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int kz = q >> lt, c = q & (T - 1);
    if (c < nc) {
      const double2 g = a.Gq[(size_t)kz * nkx + kx0 + c];
      lds[c * M + bitrev(kz, bits)] = make_double2(g.x, -g.y);
    }
  }
  for (int m = threadIdx.x; m < M / 2; m += blockDim.x) tws[m] = a.tw[R.Lx + m];
  lds_fft(lds, bits, nc, tws);
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int j = q >> lt, c = q & (T - 1);
    if (c >= nc) continue;
    const double2 v = lds[c * M + j];
    a.rows[(size_t)j * nkx + kx0 + c] = make_double2(v.x, -v.y);
  }
}

// one block per row j: adjfield(x, j) = norm Re sum_{kx <= Lx/2} rows[j][kx]
// e^{+2 pi i kx x / Lx} = norm Re FFT(conj(rows[j][.]) padded with zeros)(x)
__global__ void k_adj_rows_inv_fft(const SpecArgs a) {
  extern __shared__ double2 lds[];
  const RepInfo& R = *a.rep;
  const int Lx = R.Lx, nkx = Lx / 2 + 1, bits = __ffs(Lx) - 1, j = blockIdx.x;
  double2* tws = lds + Lx;
  for (int k = threadIdx.x; k < Lx; k += blockDim.x) {
    double2 v = make_double2(0.0, 0.0);
    if (k < nkx) {
      const double2 r = a.rows[(size_t)j * nkx + k];
      v = make_double2(r.x, -r.y);
    }
    lds[bitrev(k, bits)] = v;
  }
  for (int m = threadIdx.x; m < Lx / 2; m += blockDim.x) tws[m] = a.tw[m];
  lds_fft(lds, bits, 1, tws);
  for (int x = threadIdx.x; x < Lx; x += blockDim.x)
    a.adjfield[(size_t)j * Lx + x] = lds[x].x * R.inv_norm;
}

// ---- pressure-profile misfit J = sum_j w_j (Pbar_j - P*_j)^2 ----

// One block: lam_j = dJ/d(P - P_ref)(x, j) of every node of row j in one
// sample, 2 w_j (Pbar_j - P*_j) / (n Lx), and J by a fixed-order sum.
__global__ void k_adj_pmisfit(const RepInfo* rep, const double* acc, const double* target,
                              const double* weight, double nsamp, double* lam, double* J) {
  __shared__ double sh[256];
  const RepInfo& R = *rep;
  const double* prof = acc + R.pacc_off + 2;  // sums of the row means of P - P_ref
  double part = 0;
  for (int j = threadIdx.x; j < R.Lz; j += blockDim.x) {
    const double d = prof[j] / nsamp - target[j];
    lam[j] = 2.0 * weight[j] * d / (nsamp * R.Lx);
    part += weight[j] * d * d;
  }
  sh[threadIdx.x] = part;
  for (int h = 128; h >= 1; h >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
  }
  if (threadIdx.x == 0) *J = sh[0];
}

// Pressure term of a sample step (reading R11): with lam(r) = lam_j of the
// node's row, the density adjoints adjA(r') = sum_r lam(r) dP(r)/drho^A(r')
// and adjB likewise, where P(r) = rho/3 + (G/4) sum_l w_l |c_l|^2 [rho^A(r)
// rho^B(r + c_l) + rho^B(r) rho^A(r + c_l)] and the neighbour r + c_l of a
// wall row beyond the wall is the wall row at x + c_lx.  A node r' is that
// neighbour of r = r' - c_l when that row lies in the fluid, and of
// r = (x' - c_lx, j') when r' is on a wall row and c_l points out of it.
// Also the explicit G-derivative sum_r lam(r) d(P - P_ref)(r)/dG, as one
// partial per block (components tau_s and tau_d zero).
__global__ void k_adj_psample(const RepInfo* rep, const double* dens, const double* lam,
                              double* adjfield, double* tpart) {
  __shared__ double sh[4];
  const RepInfo& R = *rep;
  const int Lx = R.Lx, Lz = R.Lz, N = Lx * Lz;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double gpart = 0;
  if (n < N) {
    const int j = n / Lx, x = n - j * Lx;
    auto rho = [&](int s, int xx, int jj) {
      xx = xx < 0 ? xx + Lx : (xx >= Lx ? xx - Lx : xx);
      jj = jj < 0 ? 0 : (jj > Lz - 1 ? Lz - 1 : jj);
      return dens[(size_t)s * N + (size_t)jj * Lx + xx];
    };
    const double G = R.G, q = 0.25 * G;
    double sA = 0, sB = 0;
    for (int l = 1; l < 9; ++l) {
      const double c2w = kWa[l] * (double)(kCXa[l] * kCXa[l] + kCZa[l] * kCZa[l]);
      sA += c2w * rho(0, x + kCXa[l], j + kCZa[l]);
      sB += c2w * rho(1, x + kCXa[l], j + kCZa[l]);
    }
    const double lam0 = lam[j];
    double gA = lam0 * (1.0 / 3.0 + q * sB);
    double gB = lam0 * (1.0 / 3.0 + q * sA);
    for (int l = 1; l < 9; ++l) {
      const double c2w = kWa[l] * (double)(kCXa[l] * kCXa[l] + kCZa[l] * kCZa[l]);
      const int js = j - kCZa[l];
      if (js >= 0 && js < Lz) {
        const double v = q * c2w * lam[js];
        gA += v * rho(1, x - kCXa[l], js);
        gB += v * rho(0, x - kCXa[l], js);
      }
      if (j + kCZa[l] < 0 || j + kCZa[l] >= Lz) {
        const double v = q * c2w * lam0;
        gA += v * rho(1, x - kCXa[l], j);
        gB += v * rho(0, x - kCXa[l], j);
      }
    }
    adjfield[n] = gA;
    adjfield[(size_t)N + n] = gB;
    const double rA = rho(0, x, j), rB = rho(1, x, j);
    gpart = lam0 * (0.25 * (rA * sB + rB * sA) - R.rho0 * R.rho0 / 12.0);
  }
  const double b = block_sum(gpart, sh);
  if (threadIdx.x == 0) tpart[3 * blockIdx.x + 2] += b;  // running G partial
}

__global__ void k_sum(const double* parts, int n, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0;
  for (int b = 0; b < n; ++b) s += parts[b];
  *out = s;
}

inline dim3 grid_for(int n) { return dim3((unsigned)((n + 255) / 256)); }

// The per-node adjoint kernels run one wavefront per block, so that lattices
// of a few tens of thousands of nodes still occupy every compute unit.
constexpr int kNodeBlock = 64;
inline dim3 node_grid(int n) { return dim3((unsigned)((n + kNodeBlock - 1) / kNodeBlock)); }

}  // namespace

hipError_t launch_adj_step(const RepInfo* d_rep, const RepInfo& h_rep, const double* state,
                           const double* mu_next, double* mu, double* dens, double* gf,
                           double* gs, const double* adjfield, int field, int64_t t,
                           double* tpart, hipStream_t s) {
  AdjArgs a{d_rep, state, mu_next, mu, dens, gf, gs, adjfield, field, t, tpart};
  const int N = h_rep.Lx * h_rep.Lz;
  const dim3 g = node_grid(N);
  hipLaunchKernelGGL(k_adj_local, g, dim3(kNodeBlock), 0, s, a);
  hipLaunchKernelGGL(k_adj_gather, g, dim3(kNodeBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adj_theta(const RepInfo& h_rep, const double* tpart, double* theta_acc,
                            hipStream_t s) {
  const int nblk = (int)node_grid(h_rep.Lx * h_rep.Lz).x;
  hipLaunchKernelGGL(k_adj_theta, dim3(1), dim3(256), 0, s, tpart, nblk, theta_acc);
  return hipGetLastError();
}

hipError_t launch_adj_pmisfit(const RepInfo* d_rep, const RepInfo& h_rep, const double* acc,
                              const double* target, const double* weight, double nsamp,
                              double* lam, double* J, hipStream_t s) {
  (void)h_rep;
  hipLaunchKernelGGL(k_adj_pmisfit, dim3(1), dim3(256), 0, s, d_rep, acc, target, weight, nsamp,
                     lam, J);
  return hipGetLastError();
}

hipError_t launch_adj_psample(const RepInfo* d_rep, const RepInfo& h_rep, const double* dens,
                              const double* lam, double* adjfield, double* tpart,
                              hipStream_t s) {
  const int N = h_rep.Lx * h_rep.Lz;
  const dim3 g = node_grid(N);
  hipLaunchKernelGGL(k_adj_psample, g, dim3(kNodeBlock), 0, s, d_rep, dens, lam, adjfield, tpart);
  return hipGetLastError();
}

hipError_t launch_sum(const double* parts, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, s, parts, n, out);
  return hipGetLastError();
}

hipError_t launch_adj_density(const RepInfo* d_rep, const RepInfo& h_rep, const double* state,
                              double* dens, hipStream_t s) {
  AdjArgs a{};
  a.rep = d_rep;
  a.state = state;
  a.dens = dens;
  hipLaunchKernelGGL(k_adj_density, node_grid(h_rep.Lx * h_rep.Lz), dim3(kNodeBlock), 0, s,
                     a);
  return hipGetLastError();
}

hipError_t launch_adj_misfit(const RepInfo* d_rep, const RepInfo& h_rep, const double2* tw,
                             const double* acc, const double* target, const double* weight,
                             double* Wq, double2* mean, double* Jpart, int field, double nsamp,
                             hipStream_t s) {
  SpecArgs a{};
  a.rep = d_rep;
  a.tw = tw;
  a.acc = acc;
  a.target = target;
  a.weight = weight;
  a.Wq = Wq;
  a.mean = mean;
  a.Jpart = Jpart;
  a.field = field;
  a.nsamp = nsamp;
  const int P = h_rep.Lz * (h_rep.Lx / 2 + 1);
  hipLaunchKernelGGL(k_adj_misfit, grid_for(P), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adj_sample(const RepInfo* d_rep, const RepInfo& h_rep, const double2* tw,
                             const double* Wq, const double2* mean, int field, double nsamp,
                             const double* dens, double2* rows, double2* Gq, double* adjfield,
                             hipStream_t s) {
  SpecArgs a{};
  a.rep = d_rep;
  a.tw = tw;
  a.Wq = const_cast<double*>(Wq);
  a.mean = const_cast<double2*>(mean);
  a.field = field;
  a.nsamp = nsamp;
  a.dens = dens;
  a.rows = rows;
  a.Gq = Gq;
  a.adjfield = adjfield;
  const int P = h_rep.Lz * (h_rep.Lx / 2 + 1), N = h_rep.Lx * h_rep.Lz;
  if (h_rep.pow2) {
    const int Lx = h_rep.Lx, Lz = h_rep.Lz, nkx = Lx / 2 + 1;
    // column tiles of 2^lt: at most 16 columns and 2048 values, and wider
    // only while at least 128 tiles remain (one sample of a small lattice
    // is latency-bound: blocks matter more than full ones)
    int lt = 0;
    while (lt < 4 && (2 << lt) * Lz <= 2048 && ((nkx + (2 << lt) - 1) >> (lt + 1)) >= 128)
      ++lt;
    const unsigned ntile = (unsigned)((nkx + (1 << lt) - 1) >> lt);
    const size_t row_lds = (size_t)(Lx + Lx / 2) * sizeof(double2);
    const size_t col_lds = (size_t)(((size_t)Lz << lt) + Lz / 2) * sizeof(double2);
    hipLaunchKernelGGL(k_adj_rows_fwd_fft, dim3(Lz), dim3(256), row_lds, s, a);
    hipLaunchKernelGGL(k_adj_cols_fwd_fft, dim3(ntile), dim3(256), col_lds, s, a, lt);
    hipLaunchKernelGGL(k_adj_cols_inv_fft, dim3(ntile), dim3(256), col_lds, s, a, lt);
    hipLaunchKernelGGL(k_adj_rows_inv_fft, dim3(Lz), dim3(256), row_lds, s, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_adj_rows_fwd, grid_for(P), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_adj_cols_fwd, grid_for(P), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_adj_cols_inv, grid_for(P), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_adj_rows_inv, grid_for(N), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace fnlb
