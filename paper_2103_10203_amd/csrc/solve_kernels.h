// Device kernels of the reduced fixed-point iteration (paper Sec. 4, steps a-d).
//
// Data held per RVE between kernels (FP32 complex):
//   coef  [C][ncoef]         strain coefficients eps^ on the half-spectrum part
//                            of the pattern (column-major: column j, rows k0 up)
//   Yc    [C][ncol][n0]      axis-0 lines of the pruned transform (column kernel)
//   Yl    [C][nlast][rows]   last-axis spectra of every row (row kernel); in 2D
//                            Yl == Yc (columns are the last-axis frequencies)
// One iteration:
//   2D: row (Yl: F -> eps -> tau -> T)   col (Yc: T -> tau^ -> Green -> eps^ -> F)
//   3D: row, mid_fwd (Yl -> Yc), col, mid_inv (Yc -> Yl)
// F carries the 1/N of the inverse DFT; every other stage is unnormalised.
#pragma once

#include "mor_internal.h"

namespace mor_k {

enum { MODE_ITER = 0, MODE_FINAL = 1, MODE_INIT = 1 };
enum { MAT_HOOKE = 0, MAT_J2 = 1 };

struct Offs {
  const int64_t* yl;     // [B] element offset of RVE b in Yl
  const int64_t* yc;     // [B] in Yc
  const int64_t* coef;   // [B] in coef / warm start
  const int64_t* field;  // [B] in field outputs and J2 state (per component plane: N)
  const int64_t* part;   // [B] in the partial-sum array (entries)
};


// Strain/stress component helpers.  2D: strain [11,22,12], stress [11,22,12,33];
// 3D: [11,22,33,23,13,12].
template <int C>
struct Comp;
template <>
struct Comp<3> {
  static constexpr int S = 4, NST = 5, NDIAG = 2;
};
template <>
struct Comp<6> {
  static constexpr int S = 6, NST = 7, NDIAG = 3;
};

// Pointwise polarisation tau = sigma(eps) - C0:eps (step a) and, if wanted,
// sigma itself and the updated J2 state.
template <int C, int MAT>
__device__ __forceinline__ void constitutive(const float* e, int ph, const MatDev& m, const float* stin, float* tau,
                                             float* sig, float* stout) {
  constexpr int ND = Comp<C>::NDIAG;
  float tr = e[0];
#pragma unroll
  for (int i = 1; i < ND; ++i) tr += e[i];
  // phase 0 or 1 (checked at plan creation): selects, not indexed loads of
  // the parameter block, and the phase differences are loop invariants
  const bool p1 = ph != 0;
  if (MAT == MAT_HOOKE) {
    const float lam = p1 ? m.lam[1] : m.lam[0], mu = p1 ? m.mu[1] : m.mu[0];
    const float dl = p1 ? m.dl[1] : m.dl[0], dm = p1 ? m.dm[1] : m.dm[0];
#pragma unroll
    for (int i = 0; i < C; ++i) tau[i] = (i < ND ? dl * tr : 0.f) + dm * e[i];
    if (sig) {
#pragma unroll
      for (int i = 0; i < C; ++i) sig[i] = (i < ND ? lam * tr : 0.f) + 2.f * mu * e[i];
      if (C == 3) sig[3] = lam * tr;
    }
  } else {
    // full 3D tensors, order 11,22,33,23,13,12
    float E[6], EP[6], alpha;
    if (C == 3) {
      E[0] = e[0]; E[1] = e[1]; E[2] = 0.f; E[3] = 0.f; E[4] = 0.f; E[5] = e[2];
      EP[0] = stin[0]; EP[1] = stin[1]; EP[2] = stin[3]; EP[3] = 0.f; EP[4] = 0.f; EP[5] = stin[2];
      alpha = stin[4];
    } else {
#pragma unroll
      for (int i = 0; i < 6; ++i) { E[i] = e[i]; EP[i] = stin[i]; }
      alpha = stin[6];
    }
    const float lam = p1 ? m.lam[1] : m.lam[0], mu = p1 ? m.mu[1] : m.mu[0];
    float ee[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) ee[i] = E[i] - EP[i];
    const float tre = ee[0] + ee[1] + ee[2];
    float st[6], s[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      st[i] = (i < 3 ? lam * tre : 0.f) + 2.f * mu * ee[i];
      s[i] = 2.f * mu * (i < 3 ? ee[i] - tre * (1.f / 3.f) : ee[i]);
    }
    const float ns = sqrtf(s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + 2.f * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]));
    const float q = 1.22474487139158905f * ns;
    const float H = p1 ? m.H[1] : m.H[0];
    const float f = q - ((p1 ? m.sy[1] : m.sy[0]) + H * alpha);
    float sg[6];
    float dg = 0.f, fac = 0.f;
    if ((p1 ? m.plastic[1] : m.plastic[0]) && f > 0.f) {
      dg = f / (3.f * mu + H);
      fac = 1.22474487139158905f * dg / ns;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) sg[i] = st[i] - 2.f * mu * fac * s[i];
    const float tr3 = E[0] + E[1] + E[2];
    if (C == 3) {
      tau[0] = sg[0] - (m.lam0 * tr3 + 2.f * m.mu0 * E[0]);
      tau[1] = sg[1] - (m.lam0 * tr3 + 2.f * m.mu0 * E[1]);
      tau[2] = sg[5] - 2.f * m.mu0 * E[5];
      if (sig) { sig[0] = sg[0]; sig[1] = sg[1]; sig[2] = sg[5]; sig[3] = sg[2]; }
      if (stout) {
        stout[0] = EP[0] + fac * s[0];
        stout[1] = EP[1] + fac * s[1];
        stout[2] = EP[5] + fac * s[5];
        stout[3] = EP[2] + fac * s[2];
        stout[4] = alpha + dg;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 6; ++i) tau[i] = sg[i] - ((i < 3 ? m.lam0 * tr3 : 0.f) + 2.f * m.mu0 * E[i]);
      if (sig) {
#pragma unroll
        for (int i = 0; i < 6; ++i) sig[i] = sg[i];
      }
      if (stout) {
#pragma unroll
        for (int i = 0; i < 6; ++i) stout[i] = EP[i] + fac * s[i];
        stout[6] = alpha + dg;
      }
    }
  }
}

// Green operator of the isotropic reference medium (Sec. 3, eq. Gamma):
// eps^ = -[(n (x) v + v (x) n)/(2 mu0) - k s n (x) n], v = tau^ n, s = n.v,
// k = (lam0 + mu0)/(mu0 (lam0 + 2 mu0)).  Applied to real and imaginary parts.
template <int C, typename T = float>
__device__ __forceinline__ void green(const T* n, const T* t, T* out, T inv_mu, T kk) {
  if (C == 3) {
    T v0 = t[0] * n[0] + t[2] * n[1];
    T v1 = t[2] * n[0] + t[1] * n[1];
    T s = n[0] * v0 + n[1] * v1;
    T ks = kk * s;
    out[0] = -(inv_mu * n[0] * v0 - ks * n[0] * n[0]);
    out[1] = -(inv_mu * n[1] * v1 - ks * n[1] * n[1]);
    out[2] = -(T(0.5) * inv_mu * (n[0] * v1 + n[1] * v0) - ks * n[0] * n[1]);
  } else {
    // t: 11,22,33,23,13,12
    T v0 = t[0] * n[0] + t[5] * n[1] + t[4] * n[2];
    T v1 = t[5] * n[0] + t[1] * n[1] + t[3] * n[2];
    T v2 = t[4] * n[0] + t[3] * n[1] + t[2] * n[2];
    T s = n[0] * v0 + n[1] * v1 + n[2] * v2;
    T ks = kk * s;
    out[0] = -(inv_mu * n[0] * v0 - ks * n[0] * n[0]);
    out[1] = -(inv_mu * n[1] * v1 - ks * n[1] * n[1]);
    out[2] = -(inv_mu * n[2] * v2 - ks * n[2] * n[2]);
    out[3] = -(T(0.5) * inv_mu * (n[1] * v2 + n[2] * v1) - ks * n[1] * n[2]);
    out[4] = -(T(0.5) * inv_mu * (n[0] * v2 + n[2] * v0) - ks * n[0] * n[2]);
    out[5] = -(T(0.5) * inv_mu * (n[0] * v1 + n[1] * v0) - ks * n[0] * n[1]);
  }
}

// Projection of a strain amplitude onto compatible strains at direction n:
// P v = Gamma^ : C0 : v = -green(n, C0 : v).  Used on warm starts.
template <int C, typename T = float, typename MT = MatDev>
__device__ __forceinline__ void project_compatible(const T* n, const T* v, T* out, const MT& m) {
  constexpr int ND = C == 3 ? 2 : 3;
  T tr = T(0);
#pragma unroll
  for (int i = 0; i < ND; ++i) tr += v[i];
  T t[C];
#pragma unroll
  for (int i = 0; i < C; ++i) t[i] = (i < ND ? m.lam0 * tr : T(0)) + T(2) * m.mu0 * v[i];
  green<C, T>(n, t, out, m.g_inv_mu0, m.g_k);
#pragma unroll
  for (int i = 0; i < C; ++i) out[i] = -out[i];
}

template <int C>
__device__ __forceinline__ float comp_weight(int c) {
  return c < Comp<C>::NDIAG ? 1.f : 2.f;  // Frobenius norm of the symmetric tensor
}

// Block reduction of one double per thread; result valid in thread 0.
__device__ __forceinline__ double block_sum_d(double v, double* lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += lds[w];
  }
  return r;
}

// Hooke law in FP64 (the FP64 path): tau = (lam - lam0) tr(eps) I + 2 (mu - mu0) eps
// and, if wanted, sigma (with sigma_33 = lam tr(eps) in plane strain).
template <int C>
__device__ __forceinline__ void hooke64(const double* e, int ph, const MatDev64& m, double* tau, double* sig) {
  constexpr int ND = Comp<C>::NDIAG;
  double tr = e[0];
#pragma unroll
  for (int i = 1; i < ND; ++i) tr += e[i];
  const bool p1 = ph != 0;
  const double dl = p1 ? m.dl[1] : m.dl[0], dm = p1 ? m.dm[1] : m.dm[0];
#pragma unroll
  for (int i = 0; i < C; ++i) tau[i] = (i < ND ? dl * tr : 0.0) + dm * e[i];
  if (sig) {
    const double lam = p1 ? m.lam[1] : m.lam[0], mu = p1 ? m.mu[1] : m.mu[0];
#pragma unroll
    for (int i = 0; i < C; ++i) sig[i] = (i < ND ? lam * tr : 0.0) + 2.0 * mu * e[i];
    if (C == 3) sig[3] = lam * tr;
  }
}

// Step a) in the precision of the generic kernels: FP32 Hooke/J2, or FP64 Hooke.
template <int C, int MAT, typename T, typename MT>
__device__ __forceinline__ void law(const T* e, int ph, const MT& m, const float* stin, T* tau, T* sig, float* stout) {
  if constexpr (sizeof(T) == sizeof(double)) {
    static_assert(MAT == MAT_HOOKE, "the FP64 path has Hooke phases only");
    hooke64<C>(e, ph, m, tau, sig);
  } else {
    constitutive<C, MAT>(e, ph, m, stin, tau, sig, stout);
  }
}

// Plan tables in the precision T of the generic kernels.
template <typename T>
struct PT;
template <>
struct PT<float> {
  __device__ static const cpx<float>* tw0(const PlanDev& P) { return P.tw0; }
  __device__ static const cpx<float>* tw1(const PlanDev& P) { return P.tw1; }
  __device__ static const cpx<float>* twh(const PlanDev& P) { return P.twh; }
  __device__ static const cpx<float>* rtw(const PlanDev& P) { return P.rtw; }
  __device__ static const float* coef_n(const PlanDev& P) { return P.coef_n; }
  __device__ static float inv_N(const PlanDev& P) { return P.inv_N; }
};
template <>
struct PT<double> {
  __device__ static const cpx<double>* tw0(const PlanDev& P) { return P.tw0_64; }
  __device__ static const cpx<double>* tw1(const PlanDev& P) { return P.tw1_64; }
  __device__ static const cpx<double>* twh(const PlanDev& P) { return P.twh_64; }
  __device__ static const cpx<double>* rtw(const PlanDev& P) { return P.rtw_64; }
  __device__ static const double* coef_n(const PlanDev& P) { return P.coef_n64; }
  __device__ static double inv_N(const PlanDev& P) { return 1.0 / (double)P.N; }
};

// ------------------------------------------------------------------ row kernel
// Workgroup = `rb` consecutive rows of one RVE.  MODE_ITER: Yl (F) -> Yl (T).
// MODE_FINAL: Yl (F) -> strain, stress fields, FP64 stress partial sums,
// committed J2 state.
template <int C, int MODE, int MAT, typename T = float, typename MT = MatDev>
__global__ __launch_bounds__(256) void k_row(const PlanDev* __restrict__ plans, const int* __restrict__ rve_list,
                                             RveState* __restrict__ st, cpx<T>* __restrict__ Yl, Offs off,
                                             MT mat, float* __restrict__ jstate, float* __restrict__ out_eps,
                                             float* __restrict__ out_sig, double* __restrict__ sig_part, int rb) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  constexpr int S = Comp<C>::S;
  constexpr int NST = Comp<C>::NST;
  const int b = rve_list[blockIdx.y];
  if (MODE == MODE_ITER && !st[b].active) return;
  const PlanDev& P = plans[st[b].plan];
  const int nh = P.nlen >> 1;
  const int rows = P.rows;
  const int r0 = blockIdx.x * rb;
  if (r0 >= rows) return;
  const int nr = min(rb, rows - r0);
  const int ss = nh + 1;
  const int nseq = C * rb;
  cpx<T>* twh = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* rtw = twh + nh;
  cpx<T>* A = rtw + nh + 1;
  cpx<T>* Bf = A + nseq * ss;
  for (int t = threadIdx.x; t < nh; t += blockDim.x) twh[t] = PT<T>::twh(P)[t];
  for (int t = threadIdx.x; t <= nh; t += blockDim.x) rtw[t] = PT<T>::rtw(P)[t];
  for (int t = threadIdx.x; t < nseq * ss; t += blockDim.x) Bf[t] = {T(0), T(0)};
  __syncthreads();
  const int nlast = P.nlast;
  cpx<T>* Y = Yl + off.yl[b];
  const int64_t cstride = (int64_t)nlast * rows;
  for (int t = threadIdx.x; t < C * nlast * nr; t += blockDim.x) {
    const int r = t % nr;
    const int q = t / nr;
    const int j = q % nlast, c = q / nlast;
    Bf[(c * rb + r) * ss + P.last_k[j]] = Y[c * cstride + (int64_t)j * rows + r0 + r];
  }
  __syncthreads();
  // pack the half spectrum X[0..nh] into a length-nh complex sequence
  for (int t = threadIdx.x; t < nseq * nh; t += blockDim.x) {
    const int q = t / nh, k = t - q * nh;
    const cpx<T> X = Bf[q * ss + k];
    const cpx<T> Xc = cconj(Bf[q * ss + nh - k]);
    const cpx<T> a = cadd(X, Xc);
    const cpx<T> dd = cmul(csub(X, Xc), cconj(rtw[k]));
    A[q * ss + k] = {a.x - dd.y, a.y + dd.x};
  }
  __syncthreads();
  cpx<T>* E = fft_stockham<T, +1>(A, Bf, nseq, ss, P.fdh, twh);
  cpx<T>* O = (E == A) ? Bf : A;

  double acc[S];
#pragma unroll
  for (int s = 0; s < S; ++s) acc[s] = 0.0;
  for (int t = threadIdx.x; t < nr * nh; t += blockDim.x) {
    const int r = t / nh, k = t - r * nh;
    const int64_t row = r0 + r;
    const uint8_t* grow = P.g + row * P.nlen;
    T e0[C], e1[C], t0[C], t1[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const cpx<T> z = E[(c * rb + r) * ss + k];
      e0[c] = z.x;
      e1[c] = z.y;
    }
    const int g0 = grow[2 * k], g1 = grow[2 * k + 1];
    if (MODE == MODE_ITER) {
      float sin0[NST], sin1[NST];
      if (MAT == MAT_J2) {
        const float* sp = jstate + off.field[b] * NST;
        const int64_t p0 = row * P.nlen + 2 * k;
#pragma unroll
        for (int i = 0; i < NST; ++i) {
          sin0[i] = sp[(int64_t)i * P.N + p0];
          sin1[i] = sp[(int64_t)i * P.N + p0 + 1];
        }
      }
      law<C, MAT>(e0, g0, mat, sin0, t0, (T*)nullptr, nullptr);
      law<C, MAT>(e1, g1, mat, sin1, t1, (T*)nullptr, nullptr);
#pragma unroll
      for (int c = 0; c < C; ++c) E[(c * rb + r) * ss + k] = {t0[c], t1[c]};
    } else {
      T s0[S], s1[S];
      float sin0[NST], sin1[NST], so0[NST], so1[NST];
      const int64_t p0 = row * P.nlen + 2 * k;
      if (MAT == MAT_J2) {
        float* sp = jstate + off.field[b] * NST;
#pragma unroll
        for (int i = 0; i < NST; ++i) {
          sin0[i] = sp[(int64_t)i * P.N + p0];
          sin1[i] = sp[(int64_t)i * P.N + p0 + 1];
        }
      }
      law<C, MAT>(e0, g0, mat, sin0, t0, s0, so0);
      law<C, MAT>(e1, g1, mat, sin1, t1, s1, so1);
      if (MAT == MAT_J2) {
        float* sp = jstate + off.field[b] * NST;
#pragma unroll
        for (int i = 0; i < NST; ++i) {
          sp[(int64_t)i * P.N + p0] = so0[i];
          sp[(int64_t)i * P.N + p0 + 1] = so1[i];
        }
      }
      if (out_eps) {
        float* fe = out_eps + off.field[b] * C;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          fe[(int64_t)c * P.N + p0] = (float)e0[c];
          fe[(int64_t)c * P.N + p0 + 1] = (float)e1[c];
        }
      }
      if (out_sig) {
        float* fs = out_sig + off.field[b] * S;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          fs[(int64_t)s * P.N + p0] = (float)s0[s];
          fs[(int64_t)s * P.N + p0 + 1] = (float)s1[s];
        }
      }
#pragma unroll
      for (int s = 0; s < S; ++s) acc[s] += (double)s0[s] + (double)s1[s];
    }
  }
  if (MODE == MODE_FINAL) {
    __shared__ double red[16];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      double v = block_sum_d(acc[s], red);
      if (threadIdx.x == 0) sig_part[(off.part[b] + blockIdx.x) * S + s] = v;
    }
    return;
  }
  __syncthreads();
  cpx<T>* Z = fft_stockham<T, -1>(E, O, nseq, ss, P.fdh, twh);
  for (int t = threadIdx.x; t < C * nlast * nr; t += blockDim.x) {
    const int r = t % nr;
    const int q = t / nr;
    const int j = q % nlast, c = q / nlast;
    const int k = P.last_k[j];
    const cpx<T>* z = Z + (c * rb + r) * ss;
    const cpx<T> Zk = z[k == nh ? 0 : k];
    const cpx<T> Zc = cconj(z[k == 0 ? 0 : nh - k]);
    const cpx<T> sm = cadd(Zk, Zc);
    const cpx<T> wd = cmul(rtw[k], csub(Zk, Zc));
    Y[c * cstride + (int64_t)j * rows + r0 + r] = {T(0.5) * (sm.x + wd.y), T(0.5) * (sm.y - wd.x)};
  }
}

// ------------------------------------------------------------------ column kernel
// Workgroup = `cb` consecutive columns of one RVE.  MODE_ITER: forward FFT
// along axis 0, Green operator on the pattern rows, residual, inverse FFT.
// MODE_INIT: coefficients from the cold or warm start, inverse FFT only.
template <int C, int MODE, typename T = float, typename MT = MatDev>
__global__ __launch_bounds__(256) void k_col(const PlanDev* __restrict__ plans, const int* __restrict__ rve_list,
                                             RveState* __restrict__ st, const double* __restrict__ ebar,
                                             cpx<T>* __restrict__ Yc, cpx<T>* __restrict__ coef,
                                             const cpx<float>* __restrict__ warm, Offs off,
                                             double* __restrict__ part, MT mat, int cb) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int b = rve_list[blockIdx.y];
  if (MODE == MODE_ITER && !st[b].active) return;
  const PlanDev& P = plans[st[b].plan];
  const int ncol = P.ncol;
  const int j0 = blockIdx.x * cb;
  if (j0 >= ncol) return;
  const int ncb = min(cb, ncol - j0);
  const int n0 = P.n0;
  const int nseq = C * cb;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* A = tw + n0;
  cpx<T>* Bf = A + nseq * n0;
  for (int t = threadIdx.x; t < n0; t += blockDim.x) tw[t] = PT<T>::tw0(P)[t];
  cpx<T>* Y = Yc + off.yc[b];
  const int64_t cstride = (int64_t)ncol * n0;
  const int ncoef = P.ncoef;
  cpx<T>* co = coef + off.coef[b];
  cpx<T>* R = A;   // forward result
  cpx<T>* O = Bf;  // zeroed buffer receiving the new coefficients
  if (MODE == MODE_ITER) {
    for (int t = threadIdx.x; t < C * ncb * n0; t += blockDim.x) {
      const int x = t % n0;
      const int q = t / n0;
      const int jj = q % ncb, c = q / ncb;
      A[(c * cb + jj) * n0 + x] = Y[c * cstride + (int64_t)(j0 + jj) * n0 + x];
    }
    __syncthreads();
    R = fft_stockham<T, -1>(A, Bf, nseq, n0, P.fd0, tw);
    O = (R == A) ? Bf : A;
  }
  for (int t = threadIdx.x; t < nseq * n0; t += blockDim.x) O[t] = {T(0), T(0)};
  __syncthreads();
    const T invN = PT<T>::inv_N(P);
  double dsum = 0.0;
  for (int jj = 0; jj < ncb; ++jj) {
    const int j = j0 + jj;
    const int kl = P.last_k[P.col_last[j]];
    const float wcol = (kl == 0 || 2 * kl == P.nlen) ? 1.f : 2.f;
    const int e1 = P.col_off[j + 1];
    for (int e = P.col_off[j] + threadIdx.x; e < e1; e += blockDim.x) {
      const int k0 = P.coef_k0[e];
      const uint8_t fl = P.coef_flag[e];
      T nr_[C], ni_[C];
      if (fl & COEF_ZERO) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
          nr_[c] = (T)((double)P.N * ebar[(int64_t)b * C + c]);
          ni_[c] = T(0);
        }
      } else if ((fl & COEF_DEAD)) {
#pragma unroll
        for (int c = 0; c < C; ++c) nr_[c] = ni_[c] = T(0);
      } else if (MODE == MODE_ITER) {
        T tr_[C], ti_[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const cpx<T> v = R[(c * cb + jj) * n0 + k0];
          tr_[c] = v.x;
          ti_[c] = v.y;
        }
        const T* cn = PT<T>::coef_n(P);
        const T nv[3] = {cn[3 * e], cn[3 * e + 1], cn[3 * e + 2]};
        green<C, T>(nv, tr_, nr_, mat.g_inv_mu0, mat.g_k);
        green<C, T>(nv, ti_, ni_, mat.g_inv_mu0, mat.g_k);
      } else {
        if (warm && st[b].warm_ok) {
          T wr[C], wi[C];
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const cpx<float> w = warm[off.coef[b] + (int64_t)c * ncoef + e];
            wr[c] = w.x;
            wi[c] = w.y;
          }
          const T* cn = PT<T>::coef_n(P);
        const T nv[3] = {cn[3 * e], cn[3 * e + 1], cn[3 * e + 2]};
          project_compatible<C, T>(nv, wr, nr_, mat);
          project_compatible<C, T>(nv, wi, ni_, mat);
        } else {
#pragma unroll
          for (int c = 0; c < C; ++c) nr_[c] = ni_[c] = T(0);
        }
      }
      if (MODE == MODE_ITER) {
        double d2 = 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const cpx<T> old = co[(int64_t)c * ncoef + e];
          const double dr = (double)nr_[c] - (double)old.x, di = (double)ni_[c] - (double)old.y;
          d2 += (double)comp_weight<C>(c) * (dr * dr + di * di);
        }
        dsum += (double)wcol * d2;
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        co[(int64_t)c * ncoef + e] = {nr_[c], ni_[c]};
        O[(c * cb + jj) * n0 + k0] = {nr_[c] * invN, ni_[c] * invN};
      }
    }
  }
  __syncthreads();
  cpx<T>* other = (O == A) ? Bf : A;
  cpx<T>* F = fft_stockham<T, +1>(O, other, nseq, n0, P.fd0, tw);
  for (int t = threadIdx.x; t < C * ncb * n0; t += blockDim.x) {
    const int x = t % n0;
    const int q = t / n0;
    const int jj = q % ncb, c = q / ncb;
    Y[c * cstride + (int64_t)(j0 + jj) * n0 + x] = F[(c * cb + jj) * n0 + x];
  }
  if (MODE == MODE_ITER) {
    __shared__ double red[16];
    const double tot = block_sum_d(dsum, red);
    if (threadIdx.x == 0) part[off.part[b] + blockIdx.x] = tot;
  }
}

// ------------------------------------------------------------------ 3D axis-1 kernels
// Workgroup = (RVE, last-axis frequency j2, block of `xb` x0 values).
// FWD: Yl lines along x1 -> FFT -> Yc at the group's columns.
// INV: Yc at the group's columns -> zero-filled line -> inverse FFT -> Yl.
template <int C, int DIR, typename T = float>
__global__ __launch_bounds__(256) void k_mid(const PlanDev* __restrict__ plans, const int* __restrict__ rve_list,
                                             RveState* __restrict__ st, cpx<T>* __restrict__ Yl,
                                             cpx<T>* __restrict__ Yc, Offs off, int xb, int check_active) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int b = rve_list[blockIdx.z];
  if (check_active && !st[b].active) return;
  const PlanDev& P = plans[st[b].plan];
  const int j2 = blockIdx.y;
  if (j2 >= P.nlast) return;
  const int n0 = P.n0, n1 = P.n1;
  const int x00 = blockIdx.x * xb;
  if (x00 >= n0) return;
  const int nx = min(xb, n0 - x00);
  const int nseq = C * xb;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* A = tw + n1;
  cpx<T>* Bf = A + nseq * n1;
  for (int t = threadIdx.x; t < n1; t += blockDim.x) tw[t] = PT<T>::tw1(P)[t];
  const int rows = P.rows;
  const int nlast = P.nlast, ncol = P.ncol;
  cpx<T>* L = Yl + off.yl[b];
  cpx<T>* Cc = Yc + off.yc[b];
  const int64_t lcs = (int64_t)nlast * rows;
  const int64_t ccs = (int64_t)ncol * n0;
  const int ja = P.last_off[j2], jb = P.last_off[j2 + 1];
  const int ng = jb - ja;
  if (DIR < 0) {
    for (int t = threadIdx.x; t < C * nx * n1; t += blockDim.x) {
      const int x1 = t % n1;
      const int q = t / n1;
      const int xi = q % nx, c = q / nx;
      A[(c * xb + xi) * n1 + x1] = L[c * lcs + (int64_t)j2 * rows + (int64_t)(x00 + xi) * n1 + x1];
    }
    __syncthreads();
    cpx<T>* R = fft_stockham<T, -1>(A, Bf, nseq, n1, P.fd1, tw);
    for (int t = threadIdx.x; t < C * ng * nx; t += blockDim.x) {
      const int xi = t % nx;
      const int q = t / nx;
      const int g = q % ng, c = q / ng;
      const int j = ja + g;
      Cc[c * ccs + (int64_t)j * n0 + x00 + xi] = R[(c * xb + xi) * n1 + P.col_k[j]];
    }
  } else {
    for (int t = threadIdx.x; t < nseq * n1; t += blockDim.x) A[t] = {T(0), T(0)};
    __syncthreads();
    for (int t = threadIdx.x; t < C * ng * nx; t += blockDim.x) {
      const int xi = t % nx;
      const int q = t / nx;
      const int g = q % ng, c = q / ng;
      const int j = ja + g;
      A[(c * xb + xi) * n1 + P.col_k[j]] = Cc[c * ccs + (int64_t)j * n0 + x00 + xi];
    }
    __syncthreads();
    cpx<T>* R = fft_stockham<T, +1>(A, Bf, nseq, n1, P.fd1, tw);
    for (int t = threadIdx.x; t < C * nx * n1; t += blockDim.x) {
      const int x1 = t % n1;
      const int q = t / n1;
      const int xi = q % nx, c = q / nx;
      L[c * lcs + (int64_t)j2 * rows + (int64_t)(x00 + xi) * n1 + x1] = R[(c * xb + xi) * n1 + x1];
    }
  }
}

// Warm-start guard: one workgroup per RVE scans its warm coefficients (the
// zero-frequency and dropped entries are not used and are skipped); a NaN or
// Inf anywhere makes the RVE start cold instead, so the iteration still runs
// from a finite compatible field.
__global__ __launch_bounds__(256) void k_warm_check(const PlanDev* __restrict__ plans,
                                                    const int* __restrict__ rve_list, int nrve,
                                                    RveState* __restrict__ st, const cpx<float>* __restrict__ warm,
                                                    Offs off, int C) {
  const int i = blockIdx.x;
  if (i >= nrve) return;
  const int b = rve_list[i];
  const PlanDev& P = plans[st[b].plan];
  const int ncoef = P.ncoef;
  const cpx<float>* w = warm + off.coef[b];
  int bad = 0;
  for (int t = threadIdx.x; t < C * ncoef; t += blockDim.x) {
    const int e = t % ncoef;
    if (P.coef_flag[e] & (COEF_ZERO | COEF_DEAD)) continue;
    const cpx<float> v = w[t];
    bad |= (isfinite(v.x) && isfinite(v.y)) ? 0 : 1;
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) st[b].warm_ok = bad ? 0 : 1;
}

// Convergence decision after a column pass (one wavefront per RVE, 4 per
// workgroup): FP64 sum of the column blocks' squared coefficient changes in a
// fixed order (lane-strided partial sums, then a butterfly over the lanes),
// Parseval residual r = sqrt(sum) / (N ||eps_bar||_F), and the stop rules.
constexpr int kConvergeRvesPerBlock = 4;
__global__ __launch_bounds__(256) void k_converge(const PlanDev* __restrict__ plans,
                                                  const int* __restrict__ rve_list, int nrve,
                                                  RveState* __restrict__ st, const double* __restrict__ part,
                                                  Offs off, int cb, unsigned int* __restrict__ active_count) {
  const int i = blockIdx.x * kConvergeRvesPerBlock + (int)(threadIdx.x >> 6);
  const int lane = (int)(threadIdx.x & 63);
  if (i >= nrve) return;  // uniform over the wavefront
  const int b = rve_list[i];
  RveState& S = st[b];
  if (!S.active) return;
  const int nblk = (plans[S.plan].ncol + cb - 1) / cb;
  double sum = 0.0;
  for (int q = lane; q < nblk; q += 64) sum += part[off.part[b] + q];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if (lane != 0) return;
  const double r = sqrt(sum) / S.denom;
  const int it = S.iters + 1;
  S.iters = it;
  S.resid = r;
  int done = 0;
  if (!(r == r) || isinf(r)) {
    S.status = MOR_E_NONFINITE;
    done = 1;
  } else if (r < S.tol) {
    S.status = MOR_OK;
    done = 1;
  } else if (it >= S.max_iter) {
    S.status = MOR_E_NOT_CONVERGED;
    done = 1;
  }
  if (done) {
    S.active = 0;
    atomicSub(active_count, 1u);
  }
}

// Per-RVE grid mean of the stress: FP64 sum of the block partials divided by
// N (paper Sec. 2, volume average).  One wavefront per (RVE, component):
// lane l sums partials l, l + 64, ... in order, then a fixed butterfly over
// the lanes, so the result does not depend on scheduling.
template <int S>
__global__ __launch_bounds__(256) void k_sig_reduce(const PlanDev* __restrict__ plans,
                                                    const RveState* __restrict__ st,
                                                    const int* __restrict__ rve_list, int nrve,
                                                    const double* __restrict__ sig_part, Offs off,
                                                    const int* __restrict__ nblk, double* __restrict__ eff,
                                                    int eff_stride) {
  const int w = (int)((blockIdx.x * blockDim.x + threadIdx.x) / 64);  // uniform per wavefront
  const int lane = threadIdx.x % 64;
  if (w >= nrve * S) return;
  const int i = w / S, s = w - i * S;
  const int b = rve_list[i];
  double acc = 0.0;
  const int nb = nblk[i];
  for (int k = lane; k < nb; k += 64) acc += sig_part[(off.part[b] + k) * S + s];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) eff[(int64_t)b * eff_stride + s] = acc / (double)plans[st[b].plan].N;
}

}  // namespace mor_k
