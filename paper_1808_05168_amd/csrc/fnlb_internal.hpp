// Internal definitions of the fnlb GPU library shared by its host runtime and
// its kernels: per-replica device tables, work-item tables, buffer layouts and
// kernel-launch entry points.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "fnlb.h"

#include <cstddef>
#include <cstdint>

namespace fnlb {

struct BmTables;  // tables of the FP64 Box-Muller (fnlb_device.hpp)

// A block of four wavefronts updates a segment of 256 consecutive columns of
// one row range.  Rows are padded to 64 elements so every segment starts on a
// cache-line boundary.
constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kSeg = kBlock;
constexpr int kRowAlign = 64;

// sampled real fields: delta c, delta rho, and U_x, U_z on request; the
// sampling step stores them per node as complex pairs (delta c, delta rho)
// [, (U_x, U_z)], the sequences the row transform takes, and sums the
// pressure deviations of each row in parts of 64 columns
__host__ __device__ inline int n_fields(int flags) { return (flags & FNLB_SAMPLE_VELOCITY) ? 4 : 2; }
// Parts of a row's pressure sum in a sample: one per 64 columns.
__host__ __device__ inline int pressure_parts(int Lx) { return (Lx + 63) >> 6; }

// Everything a kernel needs about one replica.  Filled on the host, copied to
// the work buffer once at init, read by the kernels with scalar loads.
struct alignas(256) RepInfo {
  int32_t Lx, Lz;         // lattice size
  int32_t pitch;          // row length rounded up to whole 64-column tiles (>= Lx)
  int64_t plane;          // elements per (species, link) plane
  int64_t state_off;      // element offset of this replica in one state copy
  int64_t field_off;      // element offset of the sample: pairs [1 or 2][Lz][Lx][2] (storage type)
  int64_t spec_off;       // element offset of the row spectra [2][Lz][spitch], 128-byte aligned
  int64_t acc_off;        // double offset of [2][3][Lz][Lx/2+1] sums
  int64_t pacc_off;       // double offset of {sum, sum2, profile[Lz]}
  int64_t ppart_off;      // double offset of the pressure sums [Lz][pressure_parts(Lx)]
  int64_t tw_off;         // double2 offset of twiddles: Lx entries then Lz
  int32_t flags;          // FNLB_* option bits
  int32_t pow2;           // both Lx and Lz are powers of two (FFT path)
  int32_t spitch;         // elements per row of the row spectra: Lx/2+1 rounded up to 128 B
  uint32_t seed_lo, seed_hi;
  double rho0;            // reference density rho_bar
  double grad;            // grad_c0
  double G;               // non-ideal coupling
  double ne_coef;         // grad_c0 / 3 (non-equilibrium force per density)
  double rA_mid;          // rho_bar * (1/2 - (Lz-1)/2 * grad_c0) = rho_ref^A(0)
  double rA_step;         // rho_bar * grad_c0 = rho_ref^A(j+1) - rho_ref^A(j)
  double lam[9];          // relaxation rate of each moment (lam[0] unused)
  double fac[9];          // forcing factor per moment (1 - lam/2; or 1)
  double sig[2][9];       // noise amplitudes of Eqs. (22)-(23), reference densities
  double sig_base[9];     // same without the density factor (local-noise option)
  double p_ref;           // rho_bar/3 + G rho_bar^2 / 12
  double inv_norm;        // 1 / sqrt(Lx Lz)
  const BmTables* bm;     // FP64 Box-Muller tables in the work buffer (shared)
  const void* rowc;       // per row, kRowConsts constants of a sample in the compute type
};

// Constants of row j that the sample of a node needs (formed in FP64 by
// k_row_consts, rounded once to the compute type): rho_ref^A, rho_ref^B, c_0,
// the reference parts of sum_l w_l rho^S(r + c_l) for A and B, the reference
// part of the z component of sum_l w_l c_l rho^A(r + c_l), and G/4.
constexpr int kRowConsts = 8;

// One block's work: replica, 256-column segment and a range of rows.
struct Item {
  int32_t rep, strip, j0, j1;  // strip = segment index; rows j0 .. j1 - 1
  int32_t dir;                 // marching direction along z: +1 up, -1 down
};

// A row of one replica (row transform of the structure factor).
struct RowRef {
  int32_t rep, j0, nrows, pad;  // rows j0 .. j0 + nrows - 1 of one replica
};

// A tile of k_x columns of one field of one replica (column transform).
struct ColRef {
  int32_t rep, field, kx0, ncols, ltile;  // ncols <= 2^ltile columns from kx0
};

// Wavefront transforms (sequences of 8 to 512 points): a wavefront's rows
// j0 .. j0 + nrows - 1 of one replica (nrows <= 2 x 512 / Lx for float pairs,
// 512 / Lx for double pairs), and a block's tile
// of ncols <= 2048 / Lz k_x columns of one field.
struct RowTask {
  int32_t rep, j0, nrows, pad;
};
struct ColTask {
  int32_t rep, field, kx0, ncols;
};

// Kernel modes of the fused step.
enum StepMode { kStep = 0, kStepSample = 1, kSampleOnly = 2 };

// The two-step kernel (FP32-deviation storage): a block of kTBLanes lanes
// advances whole rows of up to kTBLanes columns by two time steps in one pass,
// keeping the intermediate state in LDS.  A block holds up to 8 work items of
// the same lane width (narrow lattices share a block); each marches through
// its row range with a halo of two rows on each side for the first step.
constexpr int kTBLanes = 512;
constexpr int kTBMaxSub = 8;
struct PackItem {
  int32_t nsub;    // work items in this block (1 .. kTBMaxSub)
  int32_t lwidth;  // log2 of the lanes per work item (6 .. 9)
  int32_t niter;   // loop iterations of the block (the longest item's, even)
  int32_t pad;
  int32_t rep[kTBMaxSub], j0[kTBMaxSub], j1[kTBMaxSub], dir[kTBMaxSub];
};

struct Step2Args {
  const RepInfo* reps;
  const PackItem* items;
  int32_t n_items;
  int32_t n_blocks;       // blocks launched (multiple of 8 for the XCD map)
  const void* state_in;   // state at t
  void* state_out;        // state at t + 2
  const int64_t* t_base;  // device time counter
  int64_t t_off;          // time of the first step = *t_base + t_off
  void* fields;           // sample of f(t) (sampling mode)
  double* ppart;          // its pressure sums, [Lz][pressure_parts(Lx)] per replica
  int32_t* watchdog;      // set non-zero when a sample sees a bad state
};
hipError_t launch_step2(int mode, const Step2Args& a, hipStream_t stream);

struct StepArgs {
  const RepInfo* reps;
  const Item* items;
  int32_t n_items;
  int32_t n_blocks;       // blocks launched (multiple of 8 for the XCD map)
  int32_t chunk_rows;     // rows per work item (FP64: >= 4 reads the tables from LDS)
  const void* state_in;   // current state copy
  void* state_out;        // next state copy
  const int64_t* t_base;  // device time counter (graph replays advance it)
  int64_t t_off;          // time = *t_base + t_off
  void* fields;           // sample (float for FP32-deviation storage, else double)
  double* ppart;          // its pressure sums, [Lz][pressure_parts(Lx)] per replica
  int32_t* watchdog;      // set non-zero when a sample sees a bad state
  // FP64, one replica, or null: the full densities of the pulled input state,
  // [species][Lz][Lx] (what the adjoint of the step reads)
  double* dens;
};

// Launchers (asynchronous on `stream`).
hipError_t launch_step(int precision, int mode, const StepArgs& a, hipStream_t stream);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t stream);
hipError_t launch_twiddles(const RepInfo* d_reps, const RepInfo* h_reps, int n_rep,
                           double2* tw_base, hipStream_t stream);
// the per-row sample constants of every replica (into each RepInfo::rowc)
hipError_t launch_row_consts(const RepInfo* d_reps, const RepInfo* h_reps, int n_rep,
                             int precision, hipStream_t stream);
// Row passes of one sample into the spectrum slot spec.  The row spectra hold
// complex pairs of the storage type: double2 for FP64, float2 for
// FP32-deviation storage; spec_off, spitch and slot strides count such
// elements.
hipError_t launch_row_transform(const RepInfo* reps, const RowRef* rows, int n_rows,
                                int n_pairs, int max_row_lds, int precision, const void* fields,
                                void* spec, const double2* tw, hipStream_t stream);
// Column passes of nslots samples, slot s of the spectra and of the pressure
// sums the sampling step formed at s spec_slot and s ppart_slot elements from
// spec and ppart, added to the sums in slot order (also adds each replica's
// pressure of every sample).
hipError_t launch_col_transform(const RepInfo* reps, const ColRef* cols, int n_cols,
                                int max_lds_cols, int precision, const void* spec, int nslots,
                                size_t spec_slot, double* acc, const double2* tw,
                                const double* ppart, size_t ppart_slot, hipStream_t stream);
// the same passes for rows and columns of 8 to 512 points (powers of two)
hipError_t launch_row_fft(const RepInfo* reps, const RowTask* tasks, int n_tasks, int n_pairs,
                          int precision, const void* fields, void* spec, const double2* tw,
                          hipStream_t stream);
hipError_t launch_col_fft(const RepInfo* reps, const ColTask* tasks, int n_tasks,
                          int precision, const void* spec, int nslots, size_t spec_slot,
                          double* acc, const double2* tw, const double* ppart,
                          size_t ppart_slot, hipStream_t stream);
hipError_t launch_advance_time(int64_t* t_base, int64_t dt, hipStream_t stream);

// Adjoint of the step (single replica, FP64 storage); see k_adjoint.hip.
hipError_t launch_adj_density(const RepInfo* d_rep, const RepInfo& h_rep, const double* state,
                              double* dens, hipStream_t s);
hipError_t launch_adj_step(const RepInfo* d_rep, const RepInfo& h_rep, const double* state,
                           const double* mu_next, double* mu, double* dens, double* gf,
                           double* gs, const double* adjfield, int field, int64_t t,
                           double* tpart, hipStream_t s);
// sum of the per-block parameter partials of a reverse sweep into theta_acc
hipError_t launch_adj_theta(const RepInfo& h_rep, const double* tpart, double* theta_acc,
                            hipStream_t s);
hipError_t launch_adj_misfit(const RepInfo* d_rep, const RepInfo& h_rep, const double2* tw,
                             const double* acc, const double* target, const double* weight,
                             double* Wq, double2* mean, double* Jpart, int field, double nsamp,
                             hipStream_t s);
hipError_t launch_adj_sample(const RepInfo* d_rep, const RepInfo& h_rep, const double2* tw,
                             const double* Wq, const double2* mean, int field, double nsamp,
                             const double* dens, double2* rows, double2* Gq, double* adjfield,
                             hipStream_t s);
hipError_t launch_sum(const double* parts, int n, double* out, hipStream_t s);
// the adjoint's sample term is a pressure term instead of a structure factor
constexpr int kAdjPressure = 2;
hipError_t launch_adj_pmisfit(const RepInfo* d_rep, const RepInfo& h_rep, const double* acc,
                              const double* target, const double* weight, double nsamp,
                              double* lam, double* J, hipStream_t s);
hipError_t launch_adj_psample(const RepInfo* d_rep, const RepInfo& h_rep, const double* dens,
                              const double* lam, double* adjfield, double* tpart,
                              hipStream_t s);

}  // namespace fnlb
