// Internal structures of libmor: the device-resident plan tables, per-solve
// constants and host-side error plumbing.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/mor.h"
#include "fft_lds.h"

// ---------------------------------------------------------------- errors
void mor_set_error(const std::string& msg);

#define MOR_HIP_TRY(expr)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      mor_set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                \
      return MOR_E_DEVICE;                                                             \
    }                                                                                  \
  } while (0)

#define MOR_LAUNCH_CHECK(what)                                                         \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess) {                                                            \
      mor_set_error(std::string("launch ") + (what) + ": " + hipGetErrorString(e_));   \
      return MOR_E_DEVICE;                                                             \
    }                                                                                  \
  } while (0)

// ---------------------------------------------------------------- plan
// Coefficient flags.
enum : uint8_t { COEF_ZERO = 1, COEF_DEAD = 2 };

// Device view of a plan.  The transform is separable and pruned:
//  * the last axis (length L = nlen) is handled by the row kernel through a
//    half-length complex FFT; only the `nlast` last-axis frequencies
//    last_k[0..nlast) that occur in the half-spectrum part of the pattern
//    are kept;
//  * 3D only: axis 1 (length n1) is handled by the mid kernel, keeping per
//    last-axis frequency j2 the columns last_off[j2]..last_off[j2+1];
//  * axis 0 (length n0) is handled per "column" (a line of constant
//    trailing frequencies) by the column kernel, which also applies the
//    Green operator to the column's pattern entries
//    col_off[j]..col_off[j+1] (rows coef_k0, directions coef_n).
struct PlanDev {
  int32_t ndim, n0, n1, n2;  // n2 = 1 in 2D
  int32_t N;
  int32_t nlen;              // last-axis length (2D: n1, 3D: n2)
  int32_t rows;              // rows of the last axis (2D: n0, 3D: n0*n1)
  int32_t ncol, nlast, ncoef;
  float inv_N;
  const uint8_t* g;          // [N]
  const int32_t* col_k;      // [ncol] axis-1 frequency (3D) or last-axis frequency (2D)
  const int32_t* col_last;   // [ncol] last-axis index j2 of the column
  const int32_t* col_off;    // [ncol+1]
  const int32_t* last_k;     // [nlast] last-axis frequency of index j2
  const int32_t* last_off;   // [nlast+1] first column of group j2 (3D)
  const int32_t* coef_k0;    // [ncoef]
  const float* coef_n;       // [ncoef][3]
  const uint8_t* coef_flag;  // [ncoef]
  const cpx<float>* tw0;     // [n0]        exp(-2 pi i t/n0)
  const cpx<float>* tw1;     // [n1]        exp(-2 pi i t/n1) (3D)
  const cpx<float>* twh;     // [nlen/2]    exp(-2 pi i t/(nlen/2))
  const cpx<float>* rtw;     // [nlen]      exp(-2 pi i t/nlen)
  // FP64 copies for the FP64 solve path (same definitions, not rounded)
  const double* coef_n64;    // [ncoef][3]
  const cpx<double>* tw0_64;
  const cpx<double>* tw1_64;
  const cpx<double>* twh_64;
  const cpx<double>* rtw_64;
  FftDesc fd0, fd1, fdh;
};

struct mor_plan {
  uint64_t uid = 0;  // unique per plan in the process (caches key on it, not on the address)
  std::vector<std::pair<size_t, void*>> blocks;  // device blocks owned by the plan (pooled)
  int ndim = 0;
  int n[3] = {1, 1, 1};
  int64_t N = 0, M = 0, M_actual = 0, count = 0;
  int gamma_kind = 0;
  int pattern_kind = 0;  // MOR_PATTERN_*
  int radial_lines = 0;  // lines of a radial pattern
  int device = 0;
  // device buffers owned by the plan
  uint8_t* d_g = nullptr;
  int64_t* d_sorted = nullptr;
  int64_t* d_rank = nullptr;
  int64_t* d_coef_lin = nullptr;
  int32_t* d_ints = nullptr;     // col_k | col_last | col_off | last_k | last_off | coef_k0
  float* d_coef_n = nullptr;
  uint8_t* d_coef_flag = nullptr;
  cpx<float>* d_tw = nullptr;    // tw0 | tw1 | twh | rtw
  double* d_coef_n64 = nullptr;
  cpx<double>* d_tw64 = nullptr; // FP64 tw0 | tw1 | twh | rtw
  PlanDev* d_dev = nullptr;      // device copy of `dev`
  PlanDev dev{};
  // warm-start network tables: slot s = selected pair s+1 in rank order
  int64_t nslots = 0;
  int64_t* d_slot_rep = nullptr;     // [nslots] linear index of the pair representative
  cpx<float>* d_slot_ghat = nullptr; // [nslots] g^(rep) / inclusion count
  int32_t* d_coef_slot = nullptr;    // [ncoef] slot of the coefficient (-1: xi = 0), bit 30: conjugate member
};

// ---------------------------------------------------------------- solve
// Per-solve material constants (FP32 copies for the kernels).
// Hooke phases in FP64 (the FP64 solve path; J2 runs in FP32 only).
struct MatDev64 {
  double lam[2], mu[2];
  double lam0, mu0;
  double dl[2], dm[2];  // lam[p] - lam0 and 2 (mu[p] - mu0)
  double g_inv_mu0;     // 1/mu0
  double g_k;           // (lam0+mu0)/(mu0 (lam0+2 mu0))
};

struct MatDev {
  float lam[2], mu[2], sy[2], H[2];
  int32_t plastic[2];
  float lam0, mu0;
  float dl[2], dm[2];  // lam[p] - lam0 and 2 (mu[p] - mu0), rounded as the device would
  float g_inv_mu0;  // 1/mu0
  float g_k;        // (lam0+mu0)/(mu0 (lam0+2 mu0))
};

// Per-RVE iteration state.
struct RveState {
  int32_t active;
  int32_t iters;
  int32_t status;   // mor_status of the RVE
  int32_t plan;     // index into the plan table
  double resid;
  double denom;     // N * ||eps_bar||_F (or N when eps_bar = 0)
  double tol;
  int32_t max_iter;
  int32_t warm_ok;  // 1: the warm start (if any) is used; 0: it held a NaN/Inf and the RVE starts cold
};

// Kernel ids of the profiling counters.
enum { PK_ROW = 0, PK_COL = 1, PK_MIDF = 2, PK_MIDI = 3, PK_FINAL = 4, PK_INIT = 5, PK_COUNT = 6 };
