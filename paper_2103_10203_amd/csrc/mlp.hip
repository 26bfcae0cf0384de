// Warm-start network (an addition on top of the paper's method): a 3-layer
// perceptron x -> relu(x W1 + b1) -> relu(. W2 + b2) -> . W3 + b3 trained on
// solves of the method itself, plus the kernels that gather its inputs from a
// plan, gather its training targets from converged coefficients and scatter
// its prediction into the solver's warm-start layout.
//
// Training is FP32 (tiled register-blocked GEMMs, analytic backward, Adam);
// inference can run the same FP32 path or a BF16 MFMA GEMM with FP32
// accumulation.  All reductions are fixed-order (no float atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "mor_internal.h"

namespace {

// ------------------------------------------------------------------ FP32 GEMM
// C[m][n] = sum_k opA[m][k] opB[k][n], opA[m][k] = TA ? A[k*lda+m] : A[m*lda+k],
// opB[k][n] = TB ? B[n*ldb+k] : B[k*ldb+n].  64x64 tile, K step 16, 256
// threads, 4x4 outputs per thread.
enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_RELU = 2, EPI_RELU_MASK = 3 };

constexpr int GT = 64, GK = 16;

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A, int lda,
                                              const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                              const float* __restrict__ bias, float* __restrict__ Zout,
                                              const float* __restrict__ Zmask) {
  __shared__ float As[GK][GT + 4];
  __shared__ float Bs[GK][GT + 4];
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += GK) {
    // A tile: 64 (m) x 16 (k)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = tid + q * 256;
      int mm, kk;
      if (TA) {  // contiguous along m
        mm = t % GT;
        kk = t / GT;
      } else {  // contiguous along k
        kk = t % GK;
        mm = t / GK;
      }
      const int gm = m0 + mm, gk = k0 + kk;
      float v = 0.f;
      if (gm < M && gk < K) v = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      As[kk][mm] = v;
    }
    // B tile: 16 (k) x 64 (n)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = tid + q * 256;
      int kk, nn;
      if (TB) {  // contiguous along k
        kk = t % GK;
        nn = t / GK;
      } else {  // contiguous along n
        nn = t % GT;
        kk = t / GT;
      }
      const int gk = k0 + kk, gn = n0 + nn;
      float v = 0.f;
      if (gk < K && gn < N) v = TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      float a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + ty * 4 + i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + tx * 4 + j;
      if (gn >= N) continue;
      const int64_t o = (int64_t)gm * ldc + gn;
      float v = acc[i][j];
      if (EPI == EPI_BIAS) v += bias[gn];
      if (EPI == EPI_BIAS_RELU) {
        v += bias[gn];
        Zout[o] = v;
        v = fmaxf(v, 0.f);
      }
      if (EPI == EPI_RELU_MASK) v = Zmask[o] > 0.f ? v : 0.f;
      C[o] = v;
    }
  }
}

// ------------------------------------------------------------------ bf16 helpers
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even
  unsigned int u = __float_as_uint(f);
  unsigned int r = 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)((u + r) >> 16);
}

// ------------------------------------------------------------------ BF16 MFMA GEMM (inference)
// C[m][n] = act(sum_k A[m][k] Bt[n][k] + bias[n]) with A bf16 [M][Kp] and Bt
// bf16 [N][Kp] (K padded with zeros to a multiple of 32), FP32 accumulation
// on v_mfma_f32_32x32x16_bf16.  Workgroup = 4 wavefronts on a 128 x 128
// output tile (2 x 2 wavefronts of 64 x 64, each 2 x 2 MFMA blocks).  K is
// staged 128 at a time through LDS, the next stage's global loads issued
// before the current stage's MFMAs: at the inference batch (1024 rows) the
// grid is small, and a stage of 64 MFMAs per wavefront is what it takes to
// cover the load latency of the next one.  A last, partial stage reads zeros
// past Kp.  Output FP32 or bf16.
constexpr int MM_T = 128, MM_K = 128, MM_LD = MM_K + 8;

template <int EPI, bool OUT_BF16>
__global__ __launch_bounds__(256) void k_mm_bf16(int M, int N, int Kp, const unsigned short* __restrict__ A,
                                                 const unsigned short* __restrict__ Bt,
                                                 const float* __restrict__ bias, void* __restrict__ Cout, int ldc) {
  __shared__ __attribute__((aligned(16))) unsigned short As[MM_T][MM_LD];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[MM_T][MM_LD];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = (wave / 2) * 64, wn = (wave % 2) * 64;
  const int m0 = blockIdx.y * MM_T, n0 = blockIdx.x * MM_T;
  // staging: thread t moves 64 bf16 (eight 16-byte vectors) of A and of B:
  // row t / 2, k half (t % 2) * 64
  constexpr int SV = MM_K / 16;  // vectors per thread and matrix
  const int srow = tid / 2, sk = (tid % 2) * (MM_K / 2);
  const bool a_ok = m0 + srow < M, b_ok = n0 + srow < N;
  const uint4* ag = reinterpret_cast<const uint4*>(A + (int64_t)(m0 + srow) * Kp + sk);
  const uint4* bg = reinterpret_cast<const uint4*>(Bt + (int64_t)(n0 + srow) * Kp + sk);
  uint4 ra[SV], rb[SV];
  const uint4 z = {0u, 0u, 0u, 0u};
#define MM_FETCH(K0)                                                    \
  _Pragma("unroll") for (int q = 0; q < SV; ++q) {                      \
    /* Kp is a multiple of 8: a vector lies wholly inside or outside K */ \
    const bool kin = (K0) + sk + 8 * q < Kp;                            \
    /* plain branches, not ?: (which would select between addresses) */ \
    ra[q] = z;                                                          \
    rb[q] = z;                                                          \
    if (a_ok && kin) ra[q] = ag[(K0) / 8 + q];                          \
    if (b_ok && kin) rb[q] = bg[(K0) / 8 + q];                          \
  }
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
  MM_FETCH(0)
  for (int k0 = 0; k0 < Kp; k0 += MM_K) {
    __syncthreads();  // previous stage's fragment reads are done
#pragma unroll
    for (int q = 0; q < SV; ++q) {
      *reinterpret_cast<uint4*>(&As[srow][sk + 8 * q]) = ra[q];
      *reinterpret_cast<uint4*>(&Bs[srow][sk + 8 * q]) = rb[q];
    }
    __syncthreads();
    if (k0 + MM_K < Kp) {
      MM_FETCH(k0 + MM_K)
    }
    // gfx950's 32x32x16 bf16 MFMA: lane l holds row l % 32 and the eight
    // consecutive k (l / 32) * 8 .. + 7 of each operand
    const int r = lane % 32, kq = (lane / 32) * 8;
#pragma unroll
    for (int ks = 0; ks < MM_K; ks += 16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const bf16x8*>(&As[wm + i * 32 + r][ks + kq]);
        b[i] = *reinterpret_cast<const bf16x8*>(&Bs[wn + i * 32 + r][ks + kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
#undef MM_FETCH
  // D layout (32x32 block): lane -> column lane % 32; element e -> row
  // (e / 4) * 8 + (lane / 32) * 4 + e % 4
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gn = n0 + wn + j * 32 + lane % 32;
      if (gn >= N) continue;
      const float bb = (EPI == EPI_BIAS || EPI == EPI_BIAS_RELU) ? bias[gn] : 0.f;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int gm = m0 + wm + i * 32 + (e / 4) * 8 + (lane / 32) * 4 + e % 4;
        if (gm >= M) continue;
        float v = acc[i][j][e] + bb;
        if (EPI == EPI_BIAS_RELU) v = fmaxf(v, 0.f);
        if (OUT_BF16)
          reinterpret_cast<unsigned short*>(Cout)[(int64_t)gm * ldc + gn] = f2bf(v);
        else
          reinterpret_cast<float*>(Cout)[(int64_t)gm * ldc + gn] = v;
      }
    }
}

__global__ void k_fill_u16(unsigned short* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// dst[r][k] = bf16(src[r][k]) for k < K, zero for K <= k < Kp (row-major).
__global__ void k_rows_to_bf16(const float* __restrict__ src, int rows, int K, int Kp, unsigned short* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * Kp) return;
  const int64_t r = i / Kp;
  const int k = (int)(i - r * Kp);
  dst[i] = k < K ? f2bf(src[r * K + k]) : (unsigned short)0;
}

// Transposed bf16 weights: dst[n][k] = bf16(W[k][n]) (W row-major [K][N]),
// zero for K <= k < Kp.
__global__ void k_weight_t_bf16(const float* __restrict__ W, int K, int N, int Kp, unsigned short* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)N * Kp) return;
  const int64_t n = i / Kp;
  const int k = (int)(i - n * Kp);
  dst[i] = k < K ? f2bf(W[(int64_t)k * N + n]) : (unsigned short)0;
}

// ------------------------------------------------------------------ loss, bias grads, Adam
// dY = 2 (Y - T) / count; partial sums of (Y - T)^2 per block (FP64).
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, int64_t n, float scale,
                      float* __restrict__ dY, double* __restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    dY[i] = 2.f * d * scale;
    acc += (double)d * (double)d;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// db[n] = sum_b dZ[b][n], fixed order in FP64.
__global__ void k_colsum(const float* __restrict__ dZ, int B, int N, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double s = 0.0;
  for (int b = 0; b < B; ++b) s += dZ[(int64_t)b * N + n];
  db[n] = (float)s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------ slot kernels (2D)
struct PlanSlots {
  int32_t n0, n1, N, nslots, ncoef, count;
  const int64_t* slot_rep;
  const cpx<float>* slot_ghat;
  const int32_t* coef_slot;
  const int64_t* coef_lin;
  const float* coef_n;        // [ncoef][3] unit direction of the Green operator
  const uint8_t* coef_flag;   // [ncoef] COEF_ZERO / COEF_DEAD flags
};

// First-order (Born) term of the response, the prior the network corrects.
// With the reference medium C0 (mean Lame constants) and the cold start, the
// first iterate at xi != 0 is  eps^(xi) = -Gamma^0(n) : ((C_I - C_M) : E) g^(xi),
// so per unit macro strain e_k the response divided by N is the real 3x3
// factor r[c][k] below times g^(xi) / N.  Plane strain, components
// [11, 22, 12] (tensor shear); Gamma^0 in its isotropic closed form
// eps = -[(n v + v n) / (2 mu0) - (lam0 + mu0) / (mu0 (lam0 + 2 mu0)) (n.v) n n],
// v = tau n.
struct BornPar {
  float dlam, dmu;  // lam_I - lam_M, mu_I - mu_M
  float inv_mu0;    // 1 / mu0
  float kk;         // (lam0 + mu0) / (mu0 (lam0 + 2 mu0))
};

__device__ __forceinline__ void born_unit(float n0, float n1, const BornPar& bp, float r[3][3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float e11 = k == 0 ? 1.f : 0.f, e22 = k == 1 ? 1.f : 0.f, e12 = k == 2 ? 1.f : 0.f;
    const float t11 = bp.dlam * (e11 + e22) + 2.f * bp.dmu * e11;
    const float t22 = bp.dlam * (e11 + e22) + 2.f * bp.dmu * e22;
    const float t12 = 2.f * bp.dmu * e12;
    const float v0 = t11 * n0 + t12 * n1, v1 = t12 * n0 + t22 * n1;
    const float sv = n0 * v0 + n1 * v1;
    r[0][k] = -(n0 * v0 * bp.inv_mu0 - bp.kk * sv * n0 * n0);
    r[1][k] = -(n1 * v1 * bp.inv_mu0 - bp.kk * sv * n1 * n1);
    r[2][k] = -(0.5f * (n0 * v1 + n1 * v0) * bp.inv_mu0 - bp.kk * sv * n0 * n1);
  }
}

// Born term of coefficient e in its slot representative's frame (r g^(rep) / N),
// zero for dropped modes.  The partner's direction is -n, and Gamma^0 is even
// in n, so the factor r is the same for both members of a pair.
__device__ __forceinline__ void born_coef(const PlanSlots& P, int e, int s, const BornPar& bp, cpx<float> out[3][3]) {
  float r[3][3];
  const bool dead = P.coef_flag[e] & COEF_DEAD;
  born_unit(P.coef_n[3 * e + 0], P.coef_n[3 * e + 1], bp, r);
  const cpx<float> gh = P.slot_ghat[s];
  const float vf = (float)P.count / (float)P.N;  // g^/N = (g^/count) (count/N)
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      out[c][k] = dead ? cpx<float>{0.f, 0.f} : cpx<float>{r[c][k] * gh.x * vf, r[c][k] * gh.y * vf};
}

// X[b] = [Re g^, Im g^ (S slots), coordinates (2S), volume fraction]
__global__ void k_warm_features(const PlanSlots* __restrict__ ps, const int* __restrict__ plan_of, int B, int S,
                                float* __restrict__ X) {
  const int b = blockIdx.y;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const PlanSlots& P = ps[plan_of[b]];
  const int in = 4 * S + 1;
  float* x = X + (int64_t)b * in;
  if (s < S) {
    float gr = 0.f, gi = 0.f, c0 = 0.f, c1 = 0.f;
    if (s < P.nslots) {
      const cpx<float> gh = P.slot_ghat[s];
      gr = gh.x;
      gi = gh.y;
      const int64_t rep = P.slot_rep[s];
      const int k0 = (int)(rep / P.n1), k1 = (int)(rep % P.n1);
      const int s0 = k0 <= P.n0 / 2 ? k0 : k0 - P.n0;
      const int s1 = k1 <= P.n1 / 2 ? k1 : k1 - P.n1;
      c0 = (float)s0 / (float)P.n0;
      c1 = (float)s1 / (float)P.n1;
    }
    x[2 * s] = gr;
    x[2 * s + 1] = gi;
    x[2 * S + 2 * s] = c0;
    x[2 * S + 2 * s + 1] = c1;
  }
  if (s == 0) x[4 * S] = (float)P.count / (float)P.N;
}

// Training targets: T[b][s][c][k][re,im] = eps^_k(rep of slot s)[c] / N minus
// its Born term, from the converged coefficients of the three unit macro
// strains k (packed [B][3][C][ncoef]).  A coefficient stored as the partner of
// its slot's representative contributes its conjugate, and only when the
// representative itself is not stored.
__global__ void k_warm_targets(const PlanSlots* __restrict__ ps, const int* __restrict__ plan_of,
                               const int64_t* __restrict__ coef_base, int per_rve, int B, int S,
                               const cpx<float>* __restrict__ co,
                               BornPar bp, float* __restrict__ T) {
  const int b = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const PlanSlots& P = ps[plan_of[b]];
  if (e >= P.ncoef) return;
  const int sl = P.coef_slot[e];
  if (sl < 0) return;
  const int s = sl & ((1 << 30) - 1);
  const bool conj = (sl >> 30) & 1;
  if (s >= S) return;
  if (conj) {
    const int64_t rep = P.slot_rep[s];
    const int krep = (int)(rep % P.n1);
    if (krep <= P.n1 / 2) return;  // the representative is stored and writes
  }
  const float invN = 1.f / (float)P.N;
  cpx<float> bt[3][3];
  born_coef(P, e, s, bp, bt);
  float* t = T + (int64_t)b * (18 * S) + (int64_t)s * 18;
  for (int k = 0; k < 3; ++k) {
    for (int c = 0; c < 3; ++c) {
      cpx<float> v = co[coef_base[b] * per_rve + ((int64_t)k * 3 + c) * P.ncoef + e];
      if (conj) v.y = -v.y;
      t[(c * 3 + k) * 2] = v.x * invN - bt[c][k].x;
      t[(c * 3 + k) * 2 + 1] = v.y * invN - bt[c][k].y;
    }
  }
}

// Warm start: eps^(m)[c] = N sum_k (Born[c][k] + Y[b][s][c][k]) eps_bar[b][k]
// (conjugated for partner coefficients), Y taken as zero for slots s >= S;
// zero at xi = 0 (the solver sets the mean).
__global__ void k_warm_apply(const PlanSlots* __restrict__ ps, const int* __restrict__ plan_of,
                             const int64_t* __restrict__ coef_base, int per_rve, int B, int S,
                             const float* __restrict__ Y,
                             const double* __restrict__ ebar, BornPar bp, cpx<float>* __restrict__ warm) {
  const int b = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const PlanSlots& P = ps[plan_of[b]];
  if (e >= P.ncoef) return;
  const int sl = P.coef_slot[e];
  cpx<float> out[3] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
  if (sl >= 0) {
    const int s = sl & ((1 << 30) - 1);
    const bool conj = (sl >> 30) & 1;
    {
      // the prior covers every pair of the pattern; the network's correction
      // the first S slots
      const float* y = s < S ? Y + (int64_t)b * (18 * S) + (int64_t)s * 18 : nullptr;
      const float Nf = (float)P.N;
      cpx<float> bt[3][3];
      born_coef(P, e, s, bp, bt);
      for (int c = 0; c < 3; ++c) {
        float re = 0.f, im = 0.f;
        for (int k = 0; k < 3; ++k) {
          const float eb = (float)ebar[(int64_t)b * 3 + k];
          const float yr = y ? y[(c * 3 + k) * 2] : 0.f, yi = y ? y[(c * 3 + k) * 2 + 1] : 0.f;
          re += (yr + bt[c][k].x) * eb;
          im += (yi + bt[c][k].y) * eb;
        }
        out[c] = {re * Nf, conj ? -im * Nf : im * Nf};
      }
    }
  }
  for (int c = 0; c < 3; ++c) warm[coef_base[b] * per_rve + (int64_t)c * P.ncoef + e] = out[c];
}

}  // namespace

// ====================================================================== ABI
struct mor_mlp {
  int in = 0, hid = 0, out = 0;
  int64_t np = 0;  // parameter count
  float* p = nullptr;
  float* g = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  unsigned short* wbf = nullptr;  // bf16 transposed, K-padded copies of W1, W2, W3
  bool bf_valid = false;
  unsigned short* abf = nullptr;  // bf16 activations for inference: X | H1 | H2
  int64_t abf_cap = 0;            // rows the bf16 activation buffer holds
  int kp_in() const { return (in + 31) / 32 * 32; }
  int kp_hid() const { return (hid + 31) / 32 * 32; }
  int64_t wt1() const { return 0; }
  int64_t wt2() const { return (int64_t)hid * kp_in(); }
  int64_t wt3() const { return wt2() + (int64_t)hid * kp_hid(); }
  int64_t wt_end() const { return wt3() + (int64_t)out * kp_hid(); }
  int64_t step = 0;
  // activation workspace
  int64_t cap_b = 0;
  float* ws = nullptr;
  double* part = nullptr;
  int64_t off_W1() const { return 0; }
  int64_t off_b1() const { return (int64_t)in * hid; }
  int64_t off_W2() const { return off_b1() + hid; }
  int64_t off_b2() const { return off_W2() + (int64_t)hid * hid; }
  int64_t off_W3() const { return off_b2() + hid; }
  int64_t off_b3() const { return off_W3() + (int64_t)hid * out; }
};

namespace {

template <bool TA, bool TB, int EPI>
void gemm(hipStream_t st, int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc,
          const float* bias = nullptr, float* Z = nullptr, const float* Zm = nullptr) {
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  k_gemm<TA, TB, EPI><<<grid, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc, bias, Z, Zm);
}

mor_status mlp_reserve(mor_mlp* net, int64_t B) {
  if (B <= net->cap_b) return MOR_OK;
  (void)hipFree(net->ws);
  (void)hipFree(net->part);
  net->ws = nullptr;
  net->part = nullptr;
  // Z1 H1 Z2 H2 (B x hid each), Y dY (B x out), dH dZ (B x hid)
  const int64_t n = B * (6 * (int64_t)net->hid + 2 * (int64_t)net->out);
  if (hipMalloc((void**)&net->ws, n * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&net->part, 1024 * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    mor_set_error("mlp workspace allocation failed");
    return MOR_E_OUT_OF_MEMORY;
  }
  net->cap_b = B;
  return MOR_OK;
}

struct Act {
  float *Z1, *H1, *Z2, *H2, *Y, *dY, *dH, *dZ;
};
Act acts(mor_mlp* net, int64_t B) {
  Act a;
  float* w = net->ws;
  const int64_t h = B * net->hid, o = B * net->out;
  a.Z1 = w; w += h;
  a.H1 = w; w += h;
  a.Z2 = w; w += h;
  a.H2 = w; w += h;
  a.dH = w; w += h;
  a.dZ = w; w += h;
  a.Y = w; w += o;
  a.dY = w;
  return a;
}

void forward_fp32(mor_mlp* net, hipStream_t st, const float* X, int B, const Act& a, float* Y) {
  const float* P = net->p;
  gemm<false, false, EPI_BIAS_RELU>(st, B, net->hid, net->in, X, net->in, P + net->off_W1(), net->hid, a.H1, net->hid,
                                   P + net->off_b1(), a.Z1);
  gemm<false, false, EPI_BIAS_RELU>(st, B, net->hid, net->hid, a.H1, net->hid, P + net->off_W2(), net->hid, a.H2,
                                   net->hid, P + net->off_b2(), a.Z2);
  gemm<false, false, EPI_BIAS>(st, B, net->out, net->hid, a.H2, net->hid, P + net->off_W3(), net->out, Y, net->out,
                               P + net->off_b3());
}

// Born-term constants from the two phases (reference medium = mean Lame
// constants, as in the solver); false for NULL or non-positive-definite media.
bool born_par(const mor_phase* ph, BornPar& bp) {
  if (!ph) return false;
  const double lam0 = 0.5 * (ph[0].lambda + ph[1].lambda), mu0 = 0.5 * (ph[0].mu + ph[1].mu);
  if (!(mu0 > 0.0) || !(lam0 + mu0 > 0.0) || !std::isfinite(lam0)) return false;
  bp.dlam = (float)(ph[1].lambda - ph[0].lambda);
  bp.dmu = (float)(ph[1].mu - ph[0].mu);
  bp.inv_mu0 = (float)(1.0 / mu0);
  bp.kk = (float)((lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0)));
  return true;
}

std::vector<PlanSlots> slot_views(const mor_plan_t* plans, int64_t nplans) {
  std::vector<PlanSlots> v(nplans);
  for (int64_t i = 0; i < nplans; ++i) {
    const mor_plan* p = plans[i];
    PlanSlots& s = v[i];
    s.n0 = p->n[0];
    s.n1 = p->n[1];
    s.N = (int32_t)p->N;
    s.nslots = (int32_t)p->nslots;
    s.ncoef = p->dev.ncoef;
    s.count = (int32_t)p->count;
    s.slot_rep = p->d_slot_rep;
    s.slot_ghat = p->d_slot_ghat;
    s.coef_slot = p->d_coef_slot;
    s.coef_lin = p->d_coef_lin;
    s.coef_n = p->d_coef_n;
    s.coef_flag = p->d_coef_flag;
  }
  return v;
}

// Device copies of plan views, plan_of and per-RVE coefficient bases (in
// units of one component's coefficients), cached per (device, stream): a call
// with the same plans (by uid) and plan_of reuses them without any copy.
// A rebuild first drains the stream, since queued kernels may still read the
// old tables.
struct SlotArgs {
  std::unique_lock<std::mutex> hold;  // the stream's cache, until the launches are queued
  const PlanSlots* ps = nullptr;
  const int* po = nullptr;
  const int64_t* base = nullptr;
  int maxcoef = 0;
  double* ebar = nullptr;  // device macro strains (warm_apply)
};

struct SlotCache {
  std::mutex mu;
  std::vector<uint64_t> uids;
  std::vector<int64_t> plan_of;
  PlanSlots* ps = nullptr;
  int* po = nullptr;
  int64_t* base = nullptr;
  size_t cap_p = 0, cap_b = 0;
  int maxcoef = 0;
  std::vector<PlanSlots> h_ps;
  std::vector<int> h_po;
  std::vector<int64_t> h_base;
  double* ebar = nullptr;    // device
  double* h_ebar = nullptr;  // pinned staging of the macro strains
  size_t cap_e = 0;
  hipEvent_t ebar_done = nullptr;
};

std::mutex g_slot_mu;
std::map<std::pair<int, void*>, SlotCache*> g_slot_cache;

SlotCache* slot_cache(hipStream_t st) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_slot_mu);
  auto key = std::make_pair(dev, (void*)st);
  auto it = g_slot_cache.find(key);
  if (it != g_slot_cache.end()) return it->second;
  SlotCache* c = new SlotCache();
  g_slot_cache[key] = c;
  return c;
}

mor_status slot_args(const mor_plan_t* plans, int64_t nplans, const int64_t* plan_of, int64_t B, hipStream_t st,
                     SlotArgs& a) {
  if (!plans || nplans < 1 || !plan_of || B < 1) {
    mor_set_error("warm: invalid plans / plan_of / B");
    return MOR_E_INVALID_ARG;
  }
  for (int64_t i = 0; i < nplans; ++i) {
    if (!plans[i] || plans[i]->ndim != 2) {
      mor_set_error("warm start: 2D plans only");
      return plans[i] ? MOR_E_UNSUPPORTED : MOR_E_INVALID_ARG;
    }
  }
  for (int64_t b = 0; b < B; ++b)
    if (plan_of[b] < 0 || plan_of[b] >= nplans) {
      mor_set_error("warm: plan_of out of range");
      return MOR_E_INVALID_ARG;
    }
  SlotCache* c = slot_cache(st);
  a.hold = std::unique_lock<std::mutex>(c->mu);
  bool same = (int64_t)c->uids.size() == nplans && (int64_t)c->plan_of.size() == B;
  for (int64_t i = 0; same && i < nplans; ++i) same = c->uids[i] == plans[i]->uid;
  if (same) same = std::equal(plan_of, plan_of + B, c->plan_of.begin());
  if (!same) {
    MOR_HIP_TRY(hipStreamSynchronize(st));
    c->uids.resize(nplans);
    for (int64_t i = 0; i < nplans; ++i) c->uids[i] = plans[i]->uid;
    c->plan_of.assign(plan_of, plan_of + B);
    c->h_ps = slot_views(plans, nplans);
    c->h_po.resize(B);
    c->h_base.resize(B);
    int64_t off = 0;
    c->maxcoef = 0;
    for (int64_t b = 0; b < B; ++b) {
      c->h_po[b] = (int)plan_of[b];
      c->h_base[b] = off;
      off += c->h_ps[c->h_po[b]].ncoef;
      c->maxcoef = std::max(c->maxcoef, c->h_ps[c->h_po[b]].ncoef);
    }
    if (c->cap_p < (size_t)nplans) {
      (void)hipFree(c->ps);
      c->ps = nullptr;
      c->cap_p = 0;
      MOR_HIP_TRY(hipMalloc((void**)&c->ps, nplans * sizeof(PlanSlots)));
      c->cap_p = nplans;
    }
    if (c->cap_b < (size_t)B) {
      (void)hipFree(c->po);
      (void)hipFree(c->base);
      c->po = nullptr;
      c->base = nullptr;
      c->cap_b = 0;
      MOR_HIP_TRY(hipMalloc((void**)&c->po, B * sizeof(int)));
      MOR_HIP_TRY(hipMalloc((void**)&c->base, B * sizeof(int64_t)));
      c->cap_b = B;
    }
    MOR_HIP_TRY(hipMemcpyAsync(c->ps, c->h_ps.data(), nplans * sizeof(PlanSlots), hipMemcpyHostToDevice, st));
    MOR_HIP_TRY(hipMemcpyAsync(c->po, c->h_po.data(), B * sizeof(int), hipMemcpyHostToDevice, st));
    MOR_HIP_TRY(hipMemcpyAsync(c->base, c->h_base.data(), B * sizeof(int64_t), hipMemcpyHostToDevice, st));
    // the host vectors stay alive (and unchanged) until the next rebuild,
    // which drains the stream first
  }
  a.ps = c->ps;
  a.po = c->po;
  a.base = c->base;
  a.maxcoef = c->maxcoef;
  return MOR_OK;
}

// Macro strains of warm_apply, staged through pinned memory; the staging
// buffer is reused once the previous upload has completed.  Called with the
// stream's cache held (after slot_args).
mor_status upload_ebar(hipStream_t st, const double* host, int64_t n, SlotArgs& a) {
  SlotCache* c = slot_cache(st);
  if (c->ebar_done) MOR_HIP_TRY(hipEventSynchronize(c->ebar_done));
  if (c->cap_e < (size_t)n) {
    MOR_HIP_TRY(hipStreamSynchronize(st));
    (void)hipFree(c->ebar);
    (void)hipHostFree(c->h_ebar);
    c->ebar = nullptr;
    c->h_ebar = nullptr;
    c->cap_e = 0;
    MOR_HIP_TRY(hipMalloc((void**)&c->ebar, n * sizeof(double)));
    MOR_HIP_TRY(hipHostMalloc((void**)&c->h_ebar, n * sizeof(double), hipHostMallocDefault));
    c->cap_e = n;
  }
  if (!c->ebar_done) MOR_HIP_TRY(hipEventCreateWithFlags(&c->ebar_done, hipEventDisableTiming));
  std::memcpy(c->h_ebar, host, n * sizeof(double));
  MOR_HIP_TRY(hipMemcpyAsync(c->ebar, c->h_ebar, n * sizeof(double), hipMemcpyHostToDevice, st));
  MOR_HIP_TRY(hipEventRecord(c->ebar_done, st));
  a.ebar = c->ebar;
  return MOR_OK;
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

}  // namespace

extern "C" mor_status mor_mlp_create(int32_t in_dim, int32_t hidden, int32_t out_dim, uint64_t seed, mor_mlp_t* out) {
  if (!out || in_dim < 1 || hidden < 1 || out_dim < 1) {
    mor_set_error("mor_mlp_create: invalid sizes");
    return MOR_E_INVALID_ARG;
  }
  *out = nullptr;
  mor_mlp* net = new mor_mlp();
  net->in = in_dim;
  net->hid = hidden;
  net->out = out_dim;
  net->np = net->off_b3() + out_dim;
  const int64_t np = net->np;
  if (hipMalloc((void**)&net->p, np * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&net->g, np * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&net->m, np * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&net->v, np * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&net->wbf, net->wt_end() * sizeof(unsigned short)) != hipSuccess) {
    (void)hipGetLastError();
    mor_mlp_destroy(net);
    mor_set_error("mor_mlp_create: allocation failed");
    return MOR_E_OUT_OF_MEMORY;
  }
  // He-uniform weights, zero biases (host RNG, seeded)
  std::vector<float> h(np, 0.f);
  std::mt19937_64 rng(seed);
  auto fill = [&](int64_t off, int fi, int fo) {
    const double lim = std::sqrt(6.0 / fi);
    std::uniform_real_distribution<double> U(-lim, lim);
    for (int64_t i = 0; i < (int64_t)fi * fo; ++i) h[off + i] = (float)U(rng);
  };
  fill(net->off_W1(), in_dim, hidden);
  fill(net->off_W2(), hidden, hidden);
  fill(net->off_W3(), hidden, out_dim);
  MOR_HIP_TRY(hipMemcpy(net->p, h.data(), np * sizeof(float), hipMemcpyHostToDevice));
  MOR_HIP_TRY(hipMemset(net->m, 0, np * sizeof(float)));
  MOR_HIP_TRY(hipMemset(net->v, 0, np * sizeof(float)));
  MOR_HIP_TRY(hipMemset(net->g, 0, np * sizeof(float)));
  *out = net;
  return MOR_OK;
}

extern "C" mor_status mor_mlp_destroy(mor_mlp_t net) {
  if (!net) return MOR_OK;
  (void)hipDeviceSynchronize();
  (void)hipFree(net->p);
  (void)hipFree(net->g);
  (void)hipFree(net->m);
  (void)hipFree(net->v);
  (void)hipFree(net->abf);
  (void)hipFree(net->wbf);
  (void)hipFree(net->ws);
  (void)hipFree(net->part);
  delete net;
  return MOR_OK;
}

extern "C" mor_status mor_mlp_num_params(mor_mlp_t net, int64_t* count) {
  if (!net || !count) {
    mor_set_error("mor_mlp_num_params: NULL argument");
    return MOR_E_INVALID_ARG;
  }
  *count = net->np;
  return MOR_OK;
}

extern "C" mor_status mor_mlp_get_params(mor_mlp_t net, float* host, int64_t count, int32_t which) {
  if (!net || !host || count != net->np || which < 0 || which > 3) {
    mor_set_error("mor_mlp_get_params: invalid argument");
    return MOR_E_INVALID_ARG;
  }
  const float* src = which == 0 ? net->p : which == 1 ? net->g : which == 2 ? net->m : net->v;
  MOR_HIP_TRY(hipDeviceSynchronize());
  MOR_HIP_TRY(hipMemcpy(host, src, count * sizeof(float), hipMemcpyDeviceToHost));
  return MOR_OK;
}

extern "C" mor_status mor_mlp_set_params(mor_mlp_t net, const float* host, int64_t count, int32_t which) {
  if (!net || !host || count != net->np || which < 0 || which > 3) {
    mor_set_error("mor_mlp_set_params: invalid argument");
    return MOR_E_INVALID_ARG;
  }
  float* dst = which == 0 ? net->p : which == 1 ? net->g : which == 2 ? net->m : net->v;
  MOR_HIP_TRY(hipDeviceSynchronize());
  MOR_HIP_TRY(hipMemcpy(dst, host, count * sizeof(float), hipMemcpyHostToDevice));
  if (which == 0) net->bf_valid = false;
  return MOR_OK;
}

extern "C" mor_status mor_mlp_forward(mor_mlp_t net, const float* X, int64_t B, float* Y, int32_t precision,
                                      void* stream) {
  if (!net || !X || !Y || B < 1 || B > (1 << 24)) {
    mor_set_error("mor_mlp_forward: invalid argument");
    return MOR_E_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  mor_status s = mlp_reserve(net, B);
  if (s != MOR_OK) return s;
  Act a = acts(net, B);
  if (precision == MOR_MLP_FP32) {
    forward_fp32(net, st, X, (int)B, a, Y);
  } else if (precision == MOR_MLP_BF16) {
    // BF16 inference: transposed, K-padded bf16 weights refreshed once per
    // parameter update; activations stay bf16 between the layers
    const int kpi = net->kp_in(), kph = net->kp_hid();
    if (!net->bf_valid) {
      const int64_t n1 = (int64_t)net->hid * kpi, n2 = (int64_t)net->hid * kph, n3 = (int64_t)net->out * kph;
      k_weight_t_bf16<<<(unsigned)((n1 + 255) / 256), 256, 0, st>>>(net->p + net->off_W1(), net->in, net->hid, kpi,
                                                                   net->wbf + net->wt1());
      k_weight_t_bf16<<<(unsigned)((n2 + 255) / 256), 256, 0, st>>>(net->p + net->off_W2(), net->hid, net->hid, kph,
                                                                   net->wbf + net->wt2());
      k_weight_t_bf16<<<(unsigned)((n3 + 255) / 256), 256, 0, st>>>(net->p + net->off_W3(), net->hid, net->out, kph,
                                                                   net->wbf + net->wt3());
      MOR_LAUNCH_CHECK("weights to bf16");
      net->bf_valid = true;
    }
    if (net->abf_cap < B) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(net->abf);
      net->abf = nullptr;
      net->abf_cap = 0;
      if (hipMalloc((void**)&net->abf, (size_t)B * (kpi + 2 * kph) * sizeof(unsigned short)) != hipSuccess) {
        (void)hipGetLastError();
        mor_set_error("mor_mlp_forward: allocation failed");
        return MOR_E_OUT_OF_MEMORY;
      }
      net->abf_cap = B;
      // the K padding of H1 and H2 is never written by the GEMMs: zero it once
      const int64_t nb = (int64_t)B * (kpi + 2 * kph);
      k_fill_u16<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(net->abf, nb);
    }
    unsigned short* xb = net->abf;
    unsigned short* h1 = xb + (size_t)B * kpi;
    unsigned short* h2 = h1 + (size_t)B * kph;
    const float* P = net->p;
    const unsigned short* W = net->wbf;
    k_rows_to_bf16<<<(unsigned)((B * kpi + 255) / 256), 256, 0, st>>>(X, (int)B, net->in, kpi, xb);
    const unsigned gm = (unsigned)((B + MM_T - 1) / MM_T);
    dim3 g1((net->hid + MM_T - 1) / MM_T, gm);
    k_mm_bf16<EPI_BIAS_RELU, true><<<g1, 256, 0, st>>>((int)B, net->hid, kpi, xb, W + net->wt1(), P + net->off_b1(),
                                                       h1, kph);
    k_mm_bf16<EPI_BIAS_RELU, true><<<g1, 256, 0, st>>>((int)B, net->hid, kph, h1, W + net->wt2(), P + net->off_b2(),
                                                       h2, kph);
    dim3 g3((net->out + MM_T - 1) / MM_T, gm);
    k_mm_bf16<EPI_BIAS, false><<<g3, 256, 0, st>>>((int)B, net->out, kph, h2, W + net->wt3(), P + net->off_b3(), Y,
                                                  net->out);
  } else {
    mor_set_error("mor_mlp_forward: precision must be MOR_MLP_FP32 or MOR_MLP_BF16");
    return MOR_E_INVALID_ARG;
  }
  MOR_LAUNCH_CHECK("mlp forward");
  return MOR_OK;
}

extern "C" mor_status mor_mlp_grad(mor_mlp_t net, const float* X, const float* T, int64_t B, double* loss,
                                   void* stream) {
  if (!net || !X || !T || B < 1 || B > (1 << 24)) {
    mor_set_error("mor_mlp_grad: invalid argument");
    return MOR_E_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  mor_status s = mlp_reserve(net, B);
  if (s != MOR_OK) return s;
  Act a = acts(net, B);
  forward_fp32(net, st, X, (int)B, a, a.Y);
  const int64_t no = B * net->out;
  const int nblk = (int)std::min<int64_t>(1024, (no + 255) / 256);
  k_mse<<<nblk, 256, 0, st>>>(a.Y, T, no, 1.f / (float)no, a.dY, net->part);
  MOR_LAUNCH_CHECK("mse");
  const float* P = net->p;
  float* G = net->g;
  const int hid = net->hid, in = net->in, out = net->out, Bi = (int)B;
  // layer 3
  gemm<true, false, EPI_STORE>(st, hid, out, Bi, a.H2, hid, a.dY, out, G + net->off_W3(), out);
  k_colsum<<<(out + 255) / 256, 256, 0, st>>>(a.dY, Bi, out, G + net->off_b3());
  gemm<false, true, EPI_RELU_MASK>(st, Bi, hid, out, a.dY, out, P + net->off_W3(), out, a.dZ, hid, nullptr, nullptr,
                                   a.Z2);
  // layer 2
  gemm<true, false, EPI_STORE>(st, hid, hid, Bi, a.H1, hid, a.dZ, hid, G + net->off_W2(), hid);
  k_colsum<<<(hid + 255) / 256, 256, 0, st>>>(a.dZ, Bi, hid, G + net->off_b2());
  gemm<false, true, EPI_RELU_MASK>(st, Bi, hid, hid, a.dZ, hid, P + net->off_W2(), hid, a.dH, hid, nullptr, nullptr,
                                   a.Z1);
  // layer 1
  gemm<true, false, EPI_STORE>(st, in, hid, Bi, X, in, a.dH, hid, G + net->off_W1(), hid);
  k_colsum<<<(hid + 255) / 256, 256, 0, st>>>(a.dH, Bi, hid, G + net->off_b1());
  MOR_LAUNCH_CHECK("mlp backward");
  if (loss) {
    std::vector<double> part(nblk);
    MOR_HIP_TRY(hipMemcpyAsync(part.data(), net->part, nblk * sizeof(double), hipMemcpyDeviceToHost, st));
    MOR_HIP_TRY(hipStreamSynchronize(st));
    double tot = 0.0;
    for (double v : part) tot += v;
    *loss = tot / (double)no;
  }
  return MOR_OK;
}

extern "C" mor_status mor_mlp_adam(mor_mlp_t net, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!net || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f)) {
    mor_set_error("mor_mlp_adam: invalid argument");
    return MOR_E_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  net->step += 1;
  const float c1 = 1.f - (float)std::pow((double)beta1, (double)net->step);
  const float c2 = 1.f - (float)std::pow((double)beta2, (double)net->step);
  k_adam<<<(unsigned)((net->np + 255) / 256), 256, 0, st>>>(net->p, net->g, net->m, net->v, net->np, lr, beta1, beta2,
                                                            eps, c1, c2);
  MOR_LAUNCH_CHECK("adam");
  net->bf_valid = false;
  return MOR_OK;
}

extern "C" mor_status mor_warm_features(const mor_plan_t* plans, int64_t nplans, const int64_t* plan_of, int64_t B,
                                        int32_t nslots, float* X, void* stream) {
  if (!X || nslots < 1) {
    mor_set_error("mor_warm_features: invalid argument");
    return MOR_E_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  SlotArgs a;
  mor_status s = slot_args(plans, nplans, plan_of, B, st, a);
  if (s != MOR_OK) return s;
  dim3 grid((nslots + 255) / 256, (unsigned)B);
  k_warm_features<<<grid, 256, 0, st>>>(a.ps, a.po, (int)B, nslots, X);
  MOR_LAUNCH_CHECK("warm_features");
  return MOR_OK;
}

extern "C" mor_status mor_warm_targets(const mor_plan_t* plans, int64_t nplans, const int64_t* plan_of, int64_t B,
                                       int32_t nslots, const mor_phase phase[2], const float* coeffs, float* T,
                                       void* stream) {
  BornPar bp;
  if (!coeffs || !T || nslots < 1 || !born_par(phase, bp)) {
    mor_set_error("mor_warm_targets: invalid argument");
    return MOR_E_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  SlotArgs a;
  mor_status s = slot_args(plans, nplans, plan_of, B, st, a);
  if (s != MOR_OK) return s;
  const int64_t nt = B * 18 * (int64_t)nslots;
  k_fill_f32<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(T, nt);
  dim3 grid((a.maxcoef + 255) / 256, (unsigned)B);
  // 3 unit cases x 3 components per RVE
  k_warm_targets<<<grid, 256, 0, st>>>(a.ps, a.po, a.base, 9, (int)B, nslots, (const cpx<float>*)coeffs, bp, T);
  MOR_LAUNCH_CHECK("warm_targets");
  return MOR_OK;
}

extern "C" mor_status mor_warm_apply(const mor_plan_t* plans, int64_t nplans, const int64_t* plan_of, int64_t B,
                                     int32_t nslots, const mor_phase phase[2], const float* Y,
                                     const double* macro_strain, float* warm, void* stream) {
  BornPar bp;
  if (!Y || !macro_strain || !warm || nslots < 1 || !born_par(phase, bp)) {
    mor_set_error("mor_warm_apply: invalid argument");
    return MOR_E_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  SlotArgs a;
  mor_status s = slot_args(plans, nplans, plan_of, B, st, a);
  if (s != MOR_OK) return s;
  if ((s = upload_ebar(st, macro_strain, B * 3, a)) != MOR_OK) return s;
  dim3 grid((a.maxcoef + 255) / 256, (unsigned)B);
  k_warm_apply<<<grid, 256, 0, st>>>(a.ps, a.po, a.base, 3, (int)B, nslots, Y, a.ebar, bp, (cpx<float>*)warm);
  MOR_LAUNCH_CHECK("warm_apply");
  return MOR_OK;
}
