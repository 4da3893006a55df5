// Plain, slow, FP64 CPU oracle for the fluctuating two-species D2Q9 lattice
// Boltzmann step between two walls (Belardinelli, Sbragaglia, Benzi,
// Ciliberto, "Lattice Boltzmann Simulations of Non-Equilibrium Fluctuations
// in a Non-Ideal Binary Mixture", arXiv:1808.05168).
//
// TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU library is
// compared against.  Only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark may load it.  It shares no code, header, table or
// constant with the HIP library and must never be linked into it.
//
// Everything is written in the order and notation of the paper:
//   * lattice and moment basis ............ Sec. III, Table I, Eq. (7)
//   * LB update (collide, then stream) ..... Sec. III, Eq. (6) and Eq. (14)
//   * barycentric velocity .................. Eq. (10)
//   * non-ideal force ....................... Eq. (11)
//   * non-equilibrium acceleration .......... Eq. (12), Eq. (13) and the
//                                             footnote on a_* attached to it
//   * MRT relaxation ........................ Eq. (15), Eqs. (16)-(17)
//   * forcing moments ....................... Eq. (18) plus reading R1/R2 below
//   * thermal noise ......................... Eqs. (19)-(23)
//   * walls, periodicity, wall rules ........ Sec. III.A (Set-up)
//   * structure factor ...................... Appendix, Eqs. (A1)-(A4)
//   * pressure .............................. Eq. (24) and Sec. IV.C
//
// Where the paper leaves a choice open, the following readings are taken
// (each is listed with its reasoning in the design notes of the repository):
//   R1  first-order forcing moments carry the factor (1 - lambda_d/2), as in
//       Guo's scheme; flag ORA_FORCE_LITERAL drops it (test use only).
//   R2  higher forcing moments are Guo's: S_a = dm^eq_a/dU . F, each scaled by
//       (1 - lambda_a/2).
//   R3  the a_* correction of the footnote to Eq. (13) is on by default.
//   R4  lambda_e = lambda_Q = lambda_eps are free inputs (default 1).
//   R5  "hom" noise uses the reference densities rho_bar*c_bar0 and
//       rho_bar*(1-c_bar0); flag ORA_NOISE_LOC uses local densities instead.
//   R6  noise = Philox4x32-10 (Salmon et al., SC'11) + Box-Muller.
//   R7  wall U_z = 0: the barycentric normal momentum on a wall row is moved
//       out of the bounced-back normal population into the rest population,
//       split between species in proportion to rho^S / rho.
//   R8  ghost densities beyond the walls equal the adjacent fluid row.
//   R9  a sample of the observables is taken from f(t) before the collision of
//       step t -> t+1 whenever t >= 1 and t % sample_every == 0.
//   R11 pressure = half trace of the pressure tensor: ideal part rho/3 plus
//       the non-local interaction part (G/4) sum_l w_l |c_l|^2
//       [rho^A(r) rho^B(r+c_l) + rho^B(r) rho^A(r+c_l)].
//   R12 the z-transform runs over the L fluid rows with q_z = 2 pi k_z / L.
//   R17 the velocity fields of S_U(q) (Sec. IV.A, Eq. (31)) are the
//       barycentric U of Eq. (10) of f(t), after the wall fix, as it enters
//       the collision of the sampled step (flag ORA_VELOCITY).
//
// The simulation is a template on the scalar type so that the same code can
// be run with std::complex<double> for complex-step differentiation.  The
// Gaussian variates are plain doubles (they do not depend on parameters).

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ----------------------------------------------------------------------------
// D2Q9 lattice (Sec. III, text below Eq. (7)): velocities c_0..c_8 and weights.
// c_1 = (1,0) = -c_3, c_2 = (0,1) = -c_4, c_5 = (1,1) = -c_7, c_6 = (-1,1) = -c_8.
// ----------------------------------------------------------------------------
const int Q = 9;
const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int CZ[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const double W[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
// opposite link: c_opp(l) = -c_l
const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// Moment basis T_al of Table I and normalisations N_a = sum_l w_l T_al^2
// (Eq. (7) and the sentence after it).  Built from the definitions.
struct Basis {
  double T[Q][Q];
  double N[Q];
  Basis() {
    for (int l = 0; l < Q; ++l) {
      const double cx = CX[l], cz = CZ[l], c2 = cx * cx + cz * cz;
      T[0][l] = 1.0;
      T[1][l] = cx;
      T[2][l] = cz;
      T[3][l] = 3.0 * c2 - 2.0;
      T[4][l] = cx * cx - cz * cz;
      T[5][l] = cx * cz;
      T[6][l] = (3.0 * c2 - 4.0) * cx;
      T[7][l] = (3.0 * c2 - 4.0) * cz;
      T[8][l] = 9.0 * c2 * c2 - 15.0 * c2 + 2.0;
    }
    for (int a = 0; a < Q; ++a) {
      N[a] = 0.0;
      for (int l = 0; l < Q; ++l) N[a] += W[l] * T[a][l] * T[a][l];
    }
  }
};
const Basis B;

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): 10 rounds of a 4-word Feistel-like bijection keyed by
// a 2-word key that is bumped by two Weyl constants between rounds.
// ----------------------------------------------------------------------------
const uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
const uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                   uint32_t out[4]) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    const uint64_t p0 = (uint64_t)PHILOX_M0 * c[0];
    const uint64_t p1 = (uint64_t)PHILOX_M1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

// The 14 standard normal variates used at one node and one time step.
// 14 words per step: calls 0..2 with counter (node, t_lo, t_hi, call) give
// words 0..11; call 3 is shared by the two steps 2s and 2s + 1 (counter
// (node, 2s, 3)): step 2s takes its words 0 and 1, step 2s + 1 its words 2
// and 3, as words 12 and 13.  Key = (seed_lo, seed_hi).  Word k gives
// u_k = (w_k + 1/2) 2^-32 in (0,1); Box-Muller (Box and Muller 1958) maps the
// pair (u_2i, u_2i+1) to g_2i, g_2i+1 for i = 0..6.
void node_gaussians(uint64_t seed, uint32_t node, uint64_t t, double g[14]) {
  uint32_t words[14];
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (uint32_t call = 0; call < 3; ++call) {
    const uint32_t ctr[4] = {node, (uint32_t)t, (uint32_t)(t >> 32), call};
    philox4x32_10(ctr, key, words + 4 * call);
  }
  const uint64_t ts = t & ~(uint64_t)1;
  const uint32_t ctr3[4] = {node, (uint32_t)ts, (uint32_t)(ts >> 32), 3u};
  uint32_t shared[4];
  philox4x32_10(ctr3, key, shared);
  const int h = (int)(t & 1) * 2;
  words[12] = shared[h];
  words[13] = shared[h + 1];
  const double two_pi = 6.283185307179586476925286766559;
  for (int i = 0; i < 7; ++i) {
    const double u1 = ((double)words[2 * i] + 0.5) * 2.3283064365386962890625e-10;
    const double u2 = ((double)words[2 * i + 1] + 0.5) * 2.3283064365386962890625e-10;
    const double r = std::sqrt(-2.0 * std::log(u1));
    g[2 * i] = r * std::cos(two_pi * u2);
    g[2 * i + 1] = r * std::sin(two_pi * u2);
  }
}

}  // namespace

// ----------------------------------------------------------------------------
// Public C interface (own struct layout; mirrored by oracle.py).
// ----------------------------------------------------------------------------
extern "C" {

enum {
  ORA_ASTAR = 1,          // R3: a_* correction on
  ORA_WALL_UZ_FIX = 2,    // R7: wall U_z = 0 fix on
  ORA_NOISE_LOC = 4,      // R5: local instead of reference densities in noise
  ORA_FORCE_LITERAL = 8,  // R1: drop (1 - lambda_d/2) on first-order forcing
  ORA_VELOCITY = 32,      // also sample U_x and U_z (fields 2 and 3)
};

typedef struct {
  int32_t Lx, Lz;       // lattice: Lx periodic columns, Lz fluid rows
  double rho0;          // reference total density rho_bar
  double grad_c0;       // imposed concentration gradient
  double kT;            // thermal energy (0: noiseless)
  double G;             // non-ideal coupling
  double tau_d, tau_s, tau_e, tau_q, tau_eps;  // 1/lambda
  uint64_t seed;        // Philox key
  int32_t flags;        // ORA_* bits
  int32_t sample_every; // > 0: sample inside ora_run per reading R9
} ora_params;

}  // extern "C"

namespace {

// Parameters that may be differentiated (complex-step) are of type T.
template <typename T>
struct Theta {
  T tau_d, tau_s, G;
};

template <typename T>
struct Sim {
  const ora_params& p;
  Theta<T> th;
  int Lx, Lz;
  size_t n;  // nodes per plane

  Sim(const ora_params& pp, const Theta<T>& t) : p(pp), th(t) {
    Lx = p.Lx;
    Lz = p.Lz;
    n = (size_t)Lx * Lz;
  }

  // z coordinate of row j: walls at z = -L/2 and +L/2 sit half a link
  // outside rows 0 and L-1 (Sec. III.A, Fig. 1).
  double z_of(int j) const { return j - 0.5 * (Lz - 1); }
  // imposed background concentration c_0(z) = 1/2 + z grad_c0 (Fig. 1)
  double c0_of(int j) const { return 0.5 + z_of(j) * p.grad_c0; }

  size_t idx(int s, int l, int j, int x) const {
    return (((size_t)s * Q + l) * Lz + j) * Lx + x;
  }

  // densities rho^S = sum_l f^S_l (Eq. (8))
  void densities(const T* f, std::vector<T>& rho) const {
    rho.assign(2 * n, T(0));
    for (int s = 0; s < 2; ++s)
      for (int j = 0; j < Lz; ++j)
        for (int x = 0; x < Lx; ++x) {
          T acc = T(0);
          for (int l = 0; l < Q; ++l) acc += f[idx(s, l, j, x)];
          rho[(size_t)s * n + (size_t)j * Lx + x] = acc;
        }
  }

  // density at (x, j) with periodic x and ghost rows beyond the walls equal to
  // the adjacent fluid row (Sec. III.A, reading R8)
  T rho_at(const std::vector<T>& rho, int s, int x, int j) const {
    x = ((x % Lx) + Lx) % Lx;
    if (j < 0) j = 0;
    if (j > Lz - 1) j = Lz - 1;
    return rho[(size_t)s * n + (size_t)j * Lx + x];
  }

  // ---------------------------------------------------------------------
  // Observables of one sample (Appendix and Sec. IV.C).
  // ---------------------------------------------------------------------
  // number of sampled fields: delta c and delta rho, plus U_x and U_z when
  // the velocity structure factors are requested
  int nfields() const { return (p.flags & ORA_VELOCITY) ? 4 : 2; }

  // delta-fields: field 0 = c - c_0(z), field 1 = rho - rho_bar; with
  // ORA_VELOCITY also field 2 = U_x, field 3 = U_z (the mean velocity is zero,
  // so U itself is the fluctuation; reading R17)
  void delta_fields(const T* f, const std::vector<T>& rho, std::vector<T>& phi) const {
    phi.assign((size_t)nfields() * n, T(0));
    for (int j = 0; j < Lz; ++j)
      for (int x = 0; x < Lx; ++x) {
        const size_t k = (size_t)j * Lx + x;
        const T ra = rho[k], rb = rho[n + k];
        const T r = ra + rb;
        phi[k] = ra / r - c0_of(j);
        phi[n + k] = r - p.rho0;
        if (nfields() == 4) {
          T fl[2][Q], F[2][2], ux, uz;
          for (int s = 0; s < 2; ++s)
            for (int l = 0; l < Q; ++l) fl[s][l] = f[idx(s, l, j, x)];
          macros(rho, x, j, fl, F, ux, uz);
          phi[2 * n + k] = ux;
          phi[3 * n + k] = uz;
        }
      }
  }

  // Structure-factor sample (Appendix, Eqs. (A1)-(A4)): the discrete
  // transform Phi(q) = (Lx L)^{-1/2} sum_{x,j} dphi(x,j) e^{-i(q_x x + q_z j)}
  // with q_x = 2 pi k_x / Lx, q_z = 2 pi k_z / L (R12), done as a direct
  // separable sum (first over x for each row, then over the rows).  Real and
  // imaginary parts are kept as separate T values so that |Phi|^2 = Re^2 + Im^2
  // stays analytic for complex-step use.  Twiddle angles are reduced exactly in
  // integers.  Accumulates |Phi|^2, Re Phi, Im Phi for k_x = 0..Lx/2.
  void accumulate_sq(const std::vector<T>& phi, T* acc) const {
    const int nkx = Lx / 2 + 1;
    const double two_pi = 6.283185307179586476925286766559;
    const double norm = 1.0 / std::sqrt((double)Lx * (double)Lz);
    std::vector<double> cx(Lx), sx(Lx), cz(Lz), sz(Lz);
    for (int m = 0; m < Lx; ++m) {
      cx[m] = std::cos(two_pi * m / Lx);
      sx[m] = std::sin(two_pi * m / Lx);
    }
    for (int m = 0; m < Lz; ++m) {
      cz[m] = std::cos(two_pi * m / Lz);
      sz[m] = std::sin(two_pi * m / Lz);
    }
    const size_t plane = (size_t)Lz * nkx;
    for (int fld = 0; fld < nfields(); ++fld) {
      const T* d = phi.data() + (size_t)fld * n;
      // row transform: R(kx, j) = sum_x d(x,j) e^{-i 2 pi kx x / Lx}
      std::vector<T> rr((size_t)Lz * nkx), ri((size_t)Lz * nkx);
#pragma omp parallel for schedule(static)
      for (int j = 0; j < Lz; ++j)
        for (int kx = 0; kx < nkx; ++kx) {
          T re = T(0), im = T(0);
          for (int x = 0; x < Lx; ++x) {
            const int m = (int)(((int64_t)kx * x) % Lx);
            re += d[(size_t)j * Lx + x] * cx[m];
            im -= d[(size_t)j * Lx + x] * sx[m];
          }
          rr[(size_t)j * nkx + kx] = re;
          ri[(size_t)j * nkx + kx] = im;
        }
      // column transform: Phi(kx, kz) = sum_j R(kx, j) e^{-i 2 pi kz j / L}
      T* a2 = acc + (size_t)fld * 3 * plane;
      T* are = a2 + plane;
      T* aim = a2 + 2 * plane;
#pragma omp parallel for schedule(static)
      for (int kz = 0; kz < Lz; ++kz)
        for (int kx = 0; kx < nkx; ++kx) {
          T re = T(0), im = T(0);
          for (int j = 0; j < Lz; ++j) {
            const int m = (int)(((int64_t)kz * j) % Lz);
            const T a = rr[(size_t)j * nkx + kx], b = ri[(size_t)j * nkx + kx];
            // (a + i b)(cos - i sin)
            re += a * cz[m] + b * sz[m];
            im += b * cz[m] - a * sz[m];
          }
          re *= norm;
          im *= norm;
          const size_t o = (size_t)kz * nkx + kx;
          a2[o] += re * re + im * im;
          are[o] += re;
          aim[o] += im;
        }
    }
  }

  // Pressure sample (reading R11, reduces to Eq. (24) on a uniform state):
  // P(r) = rho/3 + (G/4) sum_{l>=1} w_l |c_l|^2 [rho^A(r) rho^B(r+c_l) +
  // rho^B(r) rho^A(r+c_l)], P_ref = rho_bar/3 + (G/12) rho_bar^2.  Adds the
  // spatial mean of P - P_ref to psum, its square to psum2, and the row means
  // to prof[j].
  void accumulate_pressure(const std::vector<T>& rho, T* psum, T* psum2,
                           T* prof) const {
    const T G = th.G;
    const T pref = p.rho0 / 3.0 + G * (p.rho0 * p.rho0 / 12.0);
    T total = T(0);
    for (int j = 0; j < Lz; ++j) {
      T row = T(0);
      for (int x = 0; x < Lx; ++x) {
        const T ra = rho_at(rho, 0, x, j), rb = rho_at(rho, 1, x, j);
        T inter = T(0);
        for (int l = 1; l < Q; ++l) {
          const double c2 = CX[l] * CX[l] + CZ[l] * CZ[l];
          inter += W[l] * c2 *
                   (ra * rho_at(rho, 1, x + CX[l], j + CZ[l]) +
                    rb * rho_at(rho, 0, x + CX[l], j + CZ[l]));
        }
        const T P = (ra + rb) / 3.0 + G * 0.25 * inter;
        row += P - pref;
      }
      if (prof) prof[j] += row / (double)Lx;
      total += row;
    }
    total /= (double)n;
    *psum += total;
    *psum2 += total * total;
  }

  // Per-node macroscopic quantities of f(t) at (x, j): force densities F^S
  // (Eqs. (11)-(13) and the a_* footnote), the wall U_z fix applied to the
  // node's populations fl (Sec. III.A, R7) and the barycentric velocity U
  // (Eq. (10)).
  void macros(const std::vector<T>& rho, int x, int j, T fl[2][Q], T F[2][2],
              T& Ux, T& Uz) const {
    const size_t k = (size_t)j * Lx + x;
    const T G = th.G;
    const double gc = p.grad_c0;
    const bool astar = (p.flags & ORA_ASTAR) != 0;
    const bool wallfix = (p.flags & ORA_WALL_UZ_FIX) != 0;
    const T rS[2] = {rho[k], rho[n + k]};
    const T r = rS[0] + rS[1];
    const T c = rS[0] / r;

    // non-ideal acceleration, Eq. (11): a^A_NI = -G sum_l w_l c_l rho^B(r+c_l)
    T sA[2] = {T(0), T(0)}, sB[2] = {T(0), T(0)};
    for (int l = 1; l < Q; ++l) {
      const T na = rho_at(rho, 0, x + CX[l], j + CZ[l]);
      const T nb = rho_at(rho, 1, x + CX[l], j + CZ[l]);
      sA[0] += W[l] * CX[l] * na;
      sA[1] += W[l] * CZ[l] * na;
      sB[0] += W[l] * CX[l] * nb;
      sB[1] += W[l] * CZ[l] * nb;
    }
    T a[2][2];  // a[s][component]
    for (int d = 0; d < 2; ++d) {
      a[0][d] = -G * sB[d];
      a[1][d] = -G * sA[d];
    }
    // a_* (footnote to Eq. (13)): a^A_* = (1-c)(a^B_NI - a^A_NI), and
    // a^B_* from rho^A a^A_* + rho^B a^B_* = 0 (Eq. (13) form).
    if (astar) {
      for (int d = 0; d < 2; ++d) {
        const T as_a = (1.0 - c) * (a[1][d] - a[0][d]);
        const T as_b = -rS[0] * as_a / rS[1];
        a[0][d] += as_a;
        a[1][d] += as_b;
      }
    }
    // non-equilibrium acceleration, Eq. (12): a^A_NE = (1/3)(0, grad_c0/c),
    // a^B_NE = (1/3)(0, grad_c0/(c-1)).
    a[0][1] += gc / (3.0 * c);
    a[1][1] += gc / (3.0 * (c - 1.0));

    // force densities F^S = rho^S a^S
    for (int s = 0; s < 2; ++s)
      for (int d = 0; d < 2; ++d) F[s][d] = rS[s] * a[s][d];

    // species momenta j^S = sum_l c_l f^S_l (Eq. (9))
    T jx[2], jz[2];
    for (int s = 0; s < 2; ++s) {
      jx[s] = T(0);
      jz[s] = T(0);
      for (int l = 0; l < Q; ++l) {
        jx[s] += (double)CX[l] * fl[s][l];
        jz[s] += (double)CZ[l] * fl[s][l];
      }
    }

    // wall rows: zero normal barycentric velocity (Sec. III.A, R7)
    if (wallfix && (j == 0 || j == Lz - 1)) {
      const T Pi = jz[0] + jz[1] + 0.5 * (F[0][1] + F[1][1]);
      for (int s = 0; s < 2; ++s) {
        const T delta = rS[s] / r * Pi;
        if (j == 0) {
          fl[s][2] -= delta;  // upward population, bounced back from below
          fl[s][0] += delta;
        } else {
          fl[s][4] += delta;  // downward population, bounced back from above
          fl[s][0] -= delta;
        }
        jz[s] -= delta;
      }
    }

    // barycentric velocity, Eq. (10): rho U = j^A + j^B + (1/2) rho a
    Ux = (jx[0] + jx[1] + 0.5 * (F[0][0] + F[1][0])) / r;
    Uz = (jz[0] + jz[1] + 0.5 * (F[0][1] + F[1][1])) / r;
  }

  // ---------------------------------------------------------------------
  // One LB time step f(t) -> f(t+1) (Eq. (6)), in place on f.
  // If sample is set, the observables of f(t) are accumulated first.
  // ---------------------------------------------------------------------
  void step(T* f, uint64_t t, bool sample, T* sq, T* psum, T* psum2, T* prof,
            int64_t* nsamp) const {
    std::vector<T> rho;
    densities(f, rho);

    if (sample) {
      std::vector<T> phi;
      delta_fields(f, rho, phi);
      if (sq) accumulate_sq(phi, sq);
      if (psum) accumulate_pressure(rho, psum, psum2, prof);
      if (nsamp) ++*nsamp;
    }

    const T lam_d = 1.0 / th.tau_d, lam_s = 1.0 / th.tau_s;
    const T lam_e = T(1.0 / p.tau_e), lam_q = T(1.0 / p.tau_q),
            lam_eps = T(1.0 / p.tau_eps);
    // relaxation rate of each moment (Table I; Eqs. (16)-(17))
    const T lam[Q] = {T(1.0), lam_d, lam_d, lam_e, lam_s,
                      lam_s,  lam_q, lam_q, lam_eps};
    const bool noise_loc = (p.flags & ORA_NOISE_LOC) != 0;
    const bool literal = (p.flags & ORA_FORCE_LITERAL) != 0;
    const double kT = p.kT;
    // reference densities of the "hom" noise (R5)
    const double rbarA = p.rho0 * 0.5, rbarB = p.rho0 * 0.5;

    std::vector<T> fout((size_t)2 * Q * n);

#pragma omp parallel for schedule(static)
    for (int j = 0; j < Lz; ++j)
      for (int x = 0; x < Lx; ++x) {
        const size_t k = (size_t)j * Lx + x;
        T fl[2][Q];
        for (int s = 0; s < 2; ++s)
          for (int l = 0; l < Q; ++l) fl[s][l] = f[idx(s, l, j, x)];
        const T rS[2] = {rho[k], rho[n + k]};
        T F[2][2], Ux, Uz;
        macros(rho, x, j, fl, F, Ux, Uz);

        // thermal noise, Eqs. (19)-(23) (diagonal in moments and space)
        double g[14];
        if (kT > 0.0) {
          node_gaussians(p.seed, (uint32_t)k, t, g);
        } else {
          for (int i = 0; i < 14; ++i) g[i] = 0.0;
        }
        const T nA = noise_loc ? rS[0] : T(rbarA);
        const T nB = noise_loc ? rS[1] : T(rbarB);
        const T sig_d = std::sqrt((2.0 - lam_d) * lam_d * kT * nA * nB / (nA + nB));
        T xi[2][Q];
        for (int s = 0; s < 2; ++s) xi[s][0] = T(0);  // Eq. (21)
        xi[0][1] = sig_d * g[0];
        xi[0][2] = sig_d * g[1];
        xi[1][1] = -xi[0][1];  // j^A_xi + j^B_xi = 0
        xi[1][2] = -xi[0][2];
        for (int aa = 3; aa < Q; ++aa) {
          xi[0][aa] = std::sqrt(3.0 * (2.0 - lam[aa]) * lam[aa] * B.N[aa] * kT * nA) *
                      g[aa - 1];
          xi[1][aa] = std::sqrt(3.0 * (2.0 - lam[aa]) * lam[aa] * B.N[aa] * kT * nB) *
                      g[aa + 5];
        }

        for (int s = 0; s < 2; ++s) {
          // moments, Eq. (7)
          T m[Q];
          for (int aa = 0; aa < Q; ++aa) {
            m[aa] = T(0);
            for (int l = 0; l < Q; ++l) m[aa] += B.T[aa][l] * fl[s][l];
          }
          // equilibrium moments m^eq(rho^S, U), Table I
          const T rs = m[0];
          T meq[Q] = {rs,
                      rs * Ux,
                      rs * Uz,
                      3.0 * rs * (Ux * Ux + Uz * Uz),
                      rs * (Ux * Ux - Uz * Uz),
                      rs * Ux * Uz,
                      T(0),
                      T(0),
                      T(0)};
          // forcing source moments (Eq. (18); readings R1, R2)
          const T Fx = F[s][0], Fz = F[s][1];
          const T Sm[Q] = {T(0),
                           Fx,
                           Fz,
                           6.0 * (Ux * Fx + Uz * Fz),
                           2.0 * (Ux * Fx - Uz * Fz),
                           Ux * Fz + Uz * Fx,
                           T(0),
                           T(0),
                           T(0)};
          // collision increment of Eq. (14): C_a + F_a + xi_a per moment
          T dm[Q];
          for (int aa = 0; aa < Q; ++aa) {
            const T C = lam[aa] * (meq[aa] - m[aa]);  // Eq. (15)
            T Fa = (1.0 - 0.5 * lam[aa]) * Sm[aa];
            if (literal && (aa == 1 || aa == 2)) Fa = Sm[aa];
            dm[aa] = C + Fa + xi[s][aa];
          }
          // R_l = w_l sum_a T_al dm_a / N_a, then f_l + R_l is streamed
          // (Eq. (6)) with mid-way bounce-back at the walls and periodic x
          // (Sec. III.A)
          for (int l = 0; l < Q; ++l) {
            T R = T(0);
            for (int aa = 0; aa < Q; ++aa) R += B.T[aa][l] * dm[aa] / B.N[aa];
            const T fs = fl[s][l] + W[l] * R;
            const int jd = j + CZ[l];
            if (jd >= 0 && jd <= Lz - 1) {
              const int xd = ((x + CX[l]) % Lx + Lx) % Lx;
              fout[idx(s, l, jd, xd)] = fs;
            } else {
              fout[idx(s, OPP[l], j, x)] = fs;
            }
          }
        }
      }
    std::memcpy((void*)f, (const void*)fout.data(), sizeof(T) * fout.size());
  }

  // Initial state (a1): f^S_l = w_l rho_0^S(z_j) with rho_0^A = rho_bar c_0(z),
  // rho_0^B = rho_bar (1 - c_0(z)) and U = 0 (Fig. 1; Sec. III.A).
  void init(T* f) const {
    for (int s = 0; s < 2; ++s)
      for (int l = 0; l < Q; ++l)
        for (int j = 0; j < Lz; ++j) {
          const double c0 = c0_of(j);
          const double rs = p.rho0 * (s == 0 ? c0 : 1.0 - c0);
          for (int x = 0; x < Lx; ++x) f[idx(s, l, j, x)] = W[l] * rs;
        }
  }

  // Run nsteps steps from time t0, sampling per reading R9.
  void run(T* f, int64_t t0, int64_t nsteps, T* sq, T* psum, T* psum2, T* prof,
           int64_t* nsamp) const {
    for (int64_t i = 0; i < nsteps; ++i) {
      const int64_t t = t0 + i;
      const bool smp = p.sample_every > 0 && t >= 1 && (t % p.sample_every) == 0;
      step(f, (uint64_t)t, smp, sq, psum, psum2, prof, nsamp);
    }
  }
};

int check_params(const ora_params* p) {
  if (!p) return -1;
  if (p->Lx < 2 || p->Lz < 2) return -1;
  if (!(p->rho0 > 0) || !(p->kT >= 0) || !(p->G >= 0)) return -1;
  const double taus[5] = {p->tau_d, p->tau_s, p->tau_e, p->tau_q, p->tau_eps};
  for (double t : taus)
    if (!(t > 0.5)) return -1;
  if (!(std::fabs(p->grad_c0) * p->Lz < 1.0)) return -1;
  return 0;
}

}  // namespace

extern "C" {

// --- unit-level entry points (used to pin the oracle against the paper) ---

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  philox4x32_10(ctr, key, out);
}

void ora_node_gaussians(uint64_t seed, uint32_t node, uint64_t t, double g[14]) {
  node_gaussians(seed, node, t, g);
}

// Export the oracle's lattice tables: c (9x2 ints as doubles), w (9),
// T (9x9, row a), N (9).
void ora_tables(double* c, double* w, double* T, double* N) {
  for (int l = 0; l < Q; ++l) {
    c[2 * l] = CX[l];
    c[2 * l + 1] = CZ[l];
    w[l] = W[l];
  }
  for (int a = 0; a < Q; ++a) {
    N[a] = B.N[a];
    for (int l = 0; l < Q; ++l) T[a * Q + l] = B.T[a][l];
  }
}

// Population form of the equilibrium moments of Table I:
// f^eq_l = w_l sum_a T_al m^eq_a(rho, U) / N_a.
void ora_equilibrium(double rho, double ux, double uz, double feq[9]) {
  const double meq[Q] = {rho,
                         rho * ux,
                         rho * uz,
                         3.0 * rho * (ux * ux + uz * uz),
                         rho * (ux * ux - uz * uz),
                         rho * ux * uz,
                         0.0,
                         0.0,
                         0.0};
  for (int l = 0; l < Q; ++l) {
    double s = 0.0;
    for (int a = 0; a < Q; ++a) s += B.T[a][l] * meq[a] / B.N[a];
    feq[l] = W[l] * s;
  }
}

// Forcing source moments S_a(U, F) used by the collision (readings R1, R2),
// before the (1 - lambda_a/2) factors.
void ora_forcing_moments(double ux, double uz, double fx, double fz, double S[9]) {
  const double Sm[Q] = {0.0, fx, fz, 6.0 * (ux * fx + uz * fz),
                        2.0 * (ux * fx - uz * fz), ux * fz + uz * fx, 0.0, 0.0, 0.0};
  for (int a = 0; a < Q; ++a) S[a] = Sm[a];
}

int ora_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void ora_set_num_threads(int nt) {
#ifdef _OPENMP
  if (nt > 0) omp_set_num_threads(nt);
#else
  (void)nt;
#endif
}

int ora_check_params(const ora_params* p) { return check_params(p); }

// --- whole-lattice entry points ---

// Layouts: f[s][l][j][x] (s = A,B; l = 0..8; j = 0..Lz-1; x = 0..Lx-1).
// sq[field][kind][kz][kx], field 0 = delta c, 1 = delta rho, and with
// ORA_VELOCITY 2 = U_x, 3 = U_z;
// kind 0 = sum |Phi|^2, 1 = sum Re Phi, 2 = sum Im Phi; kx = 0..Lx/2.
// pr = {sum_dP, sum_dP2}, prof[Lz] = sum of row means of P - P_ref.

int ora_init(const ora_params* p, double* f) {
  if (check_params(p)) return -1;
  Theta<double> th{p->tau_d, p->tau_s, p->G};
  Sim<double> sim(*p, th);
  sim.init(f);
  return 0;
}

int ora_run(const ora_params* p, int64_t t0, int64_t nsteps, double* f,
            double* sq, double* pr, double* prof, int64_t* nsamp) {
  if (check_params(p) || t0 < 0 || nsteps < 0) return -1;
  Theta<double> th{p->tau_d, p->tau_s, p->G};
  Sim<double> sim(*p, th);
  sim.run(f, t0, nsteps, sq, pr ? pr : nullptr, pr ? pr + 1 : nullptr, prof, nsamp);
  return 0;
}

// Take one sample of the current state f (no time step).
int ora_sample(const ora_params* p, const double* f, double* sq, double* pr,
               double* prof, int64_t* nsamp) {
  if (check_params(p)) return -1;
  Theta<double> th{p->tau_d, p->tau_s, p->G};
  Sim<double> sim(*p, th);
  std::vector<double> rho, phi;
  sim.densities(f, rho);
  sim.delta_fields(f, rho, phi);
  if (sq) sim.accumulate_sq(phi, sq);
  if (pr) sim.accumulate_pressure(rho, pr, pr + 1, prof);
  if (nsamp) ++*nsamp;
  return 0;
}

// Fields of the current state: rho[s][j][x] (2 planes) and
// dphi[field][j][x] (delta c, delta rho, and U_x, U_z with ORA_VELOCITY).
int ora_fields(const ora_params* p, const double* f, double* rho_out,
               double* dphi_out) {
  if (check_params(p)) return -1;
  Theta<double> th{p->tau_d, p->tau_s, p->G};
  Sim<double> sim(*p, th);
  std::vector<double> rho, phi;
  sim.densities(f, rho);
  sim.delta_fields(f, rho, phi);
  if (rho_out) std::memcpy(rho_out, rho.data(), sizeof(double) * rho.size());
  if (dphi_out) std::memcpy(dphi_out, phi.data(), sizeof(double) * phi.size());
  return 0;
}

// Barycentric velocity U[component][j][x] of the state f, after the wall fix
// (the quantity that enters the equilibrium moments of the next collision).
int ora_velocity(const ora_params* p, const double* f, double* U) {
  if (check_params(p)) return -1;
  Theta<double> th{p->tau_d, p->tau_s, p->G};
  Sim<double> sim(*p, th);
  std::vector<double> rho;
  sim.densities(f, rho);
  for (int j = 0; j < p->Lz; ++j)
    for (int x = 0; x < p->Lx; ++x) {
      double fl[2][Q], F[2][2], ux, uz;
      for (int s = 0; s < 2; ++s)
        for (int l = 0; l < Q; ++l) fl[s][l] = f[sim.idx(s, l, j, x)];
      sim.macros(rho, x, j, fl, F, ux, uz);
      U[(size_t)j * p->Lx + x] = ux;
      U[sim.n + (size_t)j * p->Lx + x] = uz;
    }
  return 0;
}

// Per-node macroscopic quantities of the state f as the collision uses them:
// the node's populations after the wall fix, fl_out[s][l][j][x] (Sec. III.A,
// R7; equal to the pulled populations off the wall rows), the force
// densities F[s][component][j][x] (Eqs. (11)-(13) with the a_* footnote) and
// the barycentric velocity U[component][j][x] (Eq. (10)).  Any output may be
// NULL.
int ora_macros(const ora_params* p, const double* f, double* fl_out, double* F_out,
               double* U_out) {
  if (check_params(p)) return -1;
  Theta<double> th{p->tau_d, p->tau_s, p->G};
  Sim<double> sim(*p, th);
  std::vector<double> rho;
  sim.densities(f, rho);
  const size_t n = sim.n;
  for (int j = 0; j < p->Lz; ++j)
    for (int x = 0; x < p->Lx; ++x) {
      const size_t k = (size_t)j * p->Lx + x;
      double fl[2][Q], F[2][2], ux, uz;
      for (int s = 0; s < 2; ++s)
        for (int l = 0; l < Q; ++l) fl[s][l] = f[sim.idx(s, l, j, x)];
      sim.macros(rho, x, j, fl, F, ux, uz);
      for (int s = 0; s < 2; ++s) {
        if (fl_out)
          for (int l = 0; l < Q; ++l) fl_out[sim.idx(s, l, j, x)] = fl[s][l];
        if (F_out)
          for (int d = 0; d < 2; ++d) F_out[(size_t)(2 * s + d) * n + k] = F[s][d];
      }
      if (U_out) {
        U_out[k] = ux;
        U_out[n + k] = uz;
      }
    }
  return 0;
}

// ---------------------------------------------------------------------------
// Structure-factor misfit over a horizon, for the gradient checks.
// From the rest state on the imposed profile at t = 0, run `horizon` steps with
// sampling per reading R9 (p->sample_every), form S(q) = <|Phi|^2> - |<Phi>|^2
// of `field` (0: delta c, 1: delta rho) over the half spectrum [k_z][k_x], and
// return J = sum_q weight_q (S(q) - S_target(q))^2.  The Gaussian variates do
// not depend on the parameters (the noise stream is held fixed).
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {
template <typename T>
T sq_misfit(const ora_params& p, const Theta<T>& th, int64_t horizon, int field,
            const double* S_target, const double* weight) {
  Sim<T> sim(p, th);
  const int nkx = p.Lx / 2 + 1;
  const size_t plane = (size_t)p.Lz * nkx;
  std::vector<T> f((size_t)2 * Q * sim.n), sq((size_t)3 * sim.nfields() * plane, T(0));
  sim.init(f.data());
  int64_t ns = 0;
  sim.run(f.data(), 0, horizon, sq.data(), nullptr, nullptr, nullptr, &ns);
  const T* a2 = sq.data() + (size_t)field * 3 * plane;
  const T* re = a2 + plane;
  const T* im = a2 + 2 * plane;
  const double n = ns > 0 ? (double)ns : 1.0;
  T J = T(0);
  for (size_t q = 0; q < plane; ++q) {
    const T mr = re[q] / n, mi = im[q] / n;
    const T S = a2[q] / n - (mr * mr + mi * mi);
    const T d = S - S_target[q];
    J += weight[q] * d * d;
  }
  return J;
}
}  // namespace

extern "C" {

int ora_sq_misfit(const ora_params* p, int64_t horizon, int field, const double* S_target,
                  const double* weight, double* J) {
  if (check_params(p) || horizon < 0 || (field != 0 && field != 1)) return -1;
  Theta<double> th{p->tau_d, p->tau_s, p->G};
  *J = sq_misfit<double>(*p, th, horizon, field, S_target, weight);
  return 0;
}

// Pressure-profile misfit over a horizon: from the rest state on the imposed
// profile, run `horizon` steps sampling the pressure per reading R9, form the
// time-averaged row means Pbar_j of P - P_ref (reading R11) and return
// J = sum_j weight_j (Pbar_j - P_target_j)^2.
}  // extern "C"

namespace {
template <typename T>
T p_misfit(const ora_params& p, const Theta<T>& th, int64_t horizon, const double* P_target,
           const double* weight) {
  Sim<T> sim(p, th);
  std::vector<T> f((size_t)2 * Q * sim.n), prof((size_t)p.Lz, T(0));
  T ps = T(0), ps2 = T(0);
  sim.init(f.data());
  int64_t ns = 0;
  sim.run(f.data(), 0, horizon, nullptr, &ps, &ps2, prof.data(), &ns);
  const double n = ns > 0 ? (double)ns : 1.0;
  T J = T(0);
  for (int j = 0; j < p.Lz; ++j) {
    const T d = prof[j] / n - P_target[j];
    J += weight[j] * d * d;
  }
  return J;
}
}  // namespace

extern "C" {

int ora_p_misfit(const ora_params* p, int64_t horizon, const double* P_target,
                 const double* weight, double* J) {
  if (check_params(p) || horizon < 0) return -1;
  Theta<double> th{p->tau_d, p->tau_s, p->G};
  *J = p_misfit<double>(*p, th, horizon, P_target, weight);
  return 0;
}

int ora_p_misfit_cs(const ora_params* p, int64_t horizon, const double* P_target,
                    const double* weight, int which, double h, double* dJ) {
  if (check_params(p) || horizon < 0 || which < 0 || which > 2 || !(h > 0)) return -1;
  typedef std::complex<double> C;
  Theta<C> th{C(p->tau_d), C(p->tau_s), C(p->G)};
  const C ih(0.0, h);
  if (which == 0) th.tau_s += ih;
  if (which == 1) th.tau_d += ih;
  if (which == 2) th.G += ih;
  const C J = p_misfit<C>(*p, th, horizon, P_target, weight);
  *dJ = J.imag() / h;
  return 0;
}

// Complex-step derivative dJ/dtheta_which (0: tau_s, 1: tau_d, 2: G):
// Im J(theta + i h e_which) / h, exact to rounding for small h.
int ora_sq_misfit_cs(const ora_params* p, int64_t horizon, int field, const double* S_target,
                     const double* weight, int which, double h, double* dJ) {
  if (check_params(p) || horizon < 0 || (field != 0 && field != 1) || which < 0 || which > 2 ||
      !(h > 0))
    return -1;
  typedef std::complex<double> C;
  Theta<C> th{C(p->tau_d), C(p->tau_s), C(p->G)};
  const C ih(0.0, h);
  if (which == 0) th.tau_s += ih;
  if (which == 1) th.tau_d += ih;
  if (which == 2) th.G += ih;
  const C J = sq_misfit<C>(*p, th, horizon, field, S_target, weight);
  *dJ = J.imag() / h;
  return 0;
}

}  // extern "C"

// The complex instantiation is what complex-step differentiation runs on.
namespace {
template struct Sim<std::complex<double>>;
}  // namespace
