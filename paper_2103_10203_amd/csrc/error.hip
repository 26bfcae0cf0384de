// Error measures of the paper's Sec. 5 for reduced solutions against a
// reference (the full set of frequencies):
//   E_bar = ||sigma_bar - sigma_bar_ref|| / ||sigma_bar_ref||,
//   E     = mean over grid points of ||sigma(x) - sigma_ref(x)|| / ||sigma_ref(x)||,
// with the Frobenius norm of the full symmetric tensor (shear components
// counted twice, sigma_33 included in plane strain).  E divides by a
// pointwise norm that may vanish: points with ||sigma_ref(x)|| <= skip_rel *
// max_x ||sigma_ref|| are left out of the mean.  Every sum is FP64 in a fixed
// order (block partials, then one wavefront per RVE), so results do not
// depend on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <map>
#include <mutex>
#include <string>

#include "mor_internal.h"

namespace {

constexpr int kErrThreads = 256;
constexpr int kErrBlocks = 128;  // blocks per RVE: fixed, so the summation order is fixed

// Squared norm of the stress at point i of one RVE's [S][N] planes.
__device__ __forceinline__ double norm2_at(const float* __restrict__ s, int64_t N, int64_t i, int S) {
  double acc = 0.0;
  for (int c = 0; c < S; ++c) {
    const double v = (double)s[c * N + i];
    // 2D [11,22,12,33]: component 2 is shear; 3D [11,22,33,23,13,12]: 3..5
    const double w = (S == 4) ? (c == 2 ? 2.0 : 1.0) : (c >= 3 ? 2.0 : 1.0);
    acc += w * v * v;
  }
  return acc;
}

__device__ __forceinline__ double norm2_diff_at(const float* __restrict__ a, const float* __restrict__ b, int64_t N,
                                                int64_t i, int S) {
  double acc = 0.0;
  for (int c = 0; c < S; ++c) {
    const double v = (double)a[c * N + i] - (double)b[c * N + i];
    const double w = (S == 4) ? (c == 2 ? 2.0 : 1.0) : (c >= 3 ? 2.0 : 1.0);
    acc += w * v * v;
  }
  return acc;
}

__global__ void k_err_clear(unsigned long long* __restrict__ rmax, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) rmax[b] = 0ull;
}

// Largest reference norm per RVE: the bit patterns of non-negative doubles
// order like their values, so an integer atomic max is exact.
__global__ __launch_bounds__(kErrThreads) void k_err_max(const float* __restrict__ ref, int64_t N, int S,
                                                        unsigned long long* __restrict__ rmax) {
  const int b = blockIdx.y;
  ref += (int64_t)b * S * N;
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, norm2_at(ref, N, i, S));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(rmax + b, (unsigned long long)__double_as_longlong(sqrt(m)));
}

// Per-block partial sums of ||sigma - sigma_ref|| / ||sigma_ref|| over the
// kept points, and their count.
__global__ __launch_bounds__(kErrThreads) void k_err_sum(const float* __restrict__ sig, const float* __restrict__ ref,
                                                        int64_t N, int S, double skip_rel,
                                                        const unsigned long long* __restrict__ rmax,
                                                        double* __restrict__ psum, double* __restrict__ pcnt) {
  __shared__ double ls[kErrThreads / 64], lc[kErrThreads / 64];
  const int b = blockIdx.y;
  sig += (int64_t)b * S * N;
  ref += (int64_t)b * S * N;
  const double thr = skip_rel * __longlong_as_double((long long)rmax[b]);
  double acc = 0.0, cnt = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const double r = sqrt(norm2_at(ref, N, i, S));
    if (r > thr) {
      acc += sqrt(norm2_diff_at(sig, ref, N, i, S)) / r;
      cnt += 1.0;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    acc += __shfl_xor(acc, o, 64);
    cnt += __shfl_xor(cnt, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    ls[w] = acc;
    lc[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, c = 0.0;
    for (int k = 0; k < kErrThreads / 64; ++k) {
      s += ls[k];
      c += lc[k];
    }
    psum[(int64_t)b * gridDim.x + blockIdx.x] = s;
    pcnt[(int64_t)b * gridDim.x + blockIdx.x] = c;
  }
}

// One wavefront per RVE: fixed-order sum of the block partials; E = 0 when
// no point is kept.
__global__ void k_err_final(const double* __restrict__ psum, const double* __restrict__ pcnt, int nblk, int B,
                            double* __restrict__ E) {
  const int b = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (b >= B) return;
  double s = 0.0, c = 0.0;
  for (int k = lane; k < nblk; k += 64) {
    s += psum[(int64_t)b * nblk + k];
    c += pcnt[(int64_t)b * nblk + k];
  }
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  if (lane == 0) E[b] = c > 0.0 ? s / c : 0.0;
}

// Device scratch of the error kernels, per device, grown on demand.
struct ErrScratch {
  void* p = nullptr;
  size_t bytes = 0;
};
std::mutex g_err_mu;
std::map<int, ErrScratch> g_err_scratch;

}  // namespace

extern "C" mor_status mor_stress_error(const float* sigma, const float* sigma_ref, const double* eff,
                                       const double* eff_ref, int64_t B, int64_t N, int32_t ndim, double skip_rel,
                                       void* stream, double* E_bar, double* E) {
  if (B < 1 || N < 1 || (ndim != 2 && ndim != 3) || !(skip_rel >= 0.0) || !std::isfinite(skip_rel)) {
    mor_set_error("mor_stress_error: need B >= 1, N >= 1, ndim 2 or 3 and a finite skip_rel >= 0");
    return MOR_E_INVALID_ARG;
  }
  if ((E && (!sigma || !sigma_ref)) || (E_bar && (!eff || !eff_ref))) {
    mor_set_error("mor_stress_error: NULL input for a requested measure");
    return MOR_E_INVALID_ARG;
  }
  const int S = ndim == 2 ? 4 : 6;
  if (E_bar) {
    for (int64_t b = 0; b < B; ++b) {
      double d2 = 0.0, r2 = 0.0;
      for (int c = 0; c < S; ++c) {
        const double w = (S == 4) ? (c == 2 ? 2.0 : 1.0) : (c >= 3 ? 2.0 : 1.0);
        const double d = eff[b * S + c] - eff_ref[b * S + c];
        d2 += w * d * d;
        r2 += w * eff_ref[b * S + c] * eff_ref[b * S + c];
      }
      E_bar[b] = r2 > 0.0 ? std::sqrt(d2 / r2) : (d2 > 0.0 ? INFINITY : 0.0);
    }
  }
  if (!E) return MOR_OK;
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  MOR_HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_err_mu);
  ErrScratch& sc = g_err_scratch[dev];
  const size_t need = (size_t)B * (8 + 2 * 8 * kErrBlocks + 8);
  if (sc.bytes < need) {
    if (sc.p) {
      MOR_HIP_TRY(hipStreamSynchronize(st));
      (void)hipFree(sc.p);
      sc.p = nullptr;
      sc.bytes = 0;
    }
    if (hipMalloc(&sc.p, need) != hipSuccess) {
      (void)hipGetLastError();
      mor_set_error("mor_stress_error: scratch allocation failed");
      return MOR_E_OUT_OF_MEMORY;
    }
    sc.bytes = need;
  }
  unsigned long long* rmax = (unsigned long long*)sc.p;
  double* psum = (double*)(rmax + B);
  double* pcnt = psum + B * kErrBlocks;
  double* dE = pcnt + B * kErrBlocks;
  const unsigned nblk = (unsigned)std::min<int64_t>(kErrBlocks, (N + kErrThreads - 1) / kErrThreads);
  k_err_clear<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(rmax, (int)B);
  MOR_LAUNCH_CHECK("err_clear");
  k_err_max<<<dim3(nblk, (unsigned)B), kErrThreads, 0, st>>>(sigma_ref, N, S, rmax);
  MOR_LAUNCH_CHECK("err_max");
  k_err_sum<<<dim3(nblk, (unsigned)B), kErrThreads, 0, st>>>(sigma, sigma_ref, N, S, skip_rel, rmax, psum, pcnt);
  MOR_LAUNCH_CHECK("err_sum");
  k_err_final<<<(unsigned)((B * 64 + 255) / 256), 256, 0, st>>>(psum, pcnt, (int)nblk, (int)B, dE);
  MOR_LAUNCH_CHECK("err_final");
  MOR_HIP_TRY(hipMemcpyAsync(E, dE, (size_t)B * sizeof(double), hipMemcpyDeviceToHost, st));
  MOR_HIP_TRY(hipStreamSynchronize(st));
  return MOR_OK;
}
