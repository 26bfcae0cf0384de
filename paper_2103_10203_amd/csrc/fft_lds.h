// Batched mixed-radix (4, 3, 2) Stockham FFT on LDS-resident sequences.
//
// A workgroup transforms `nseq` independent sequences of length n that sit in
// LDS at a + q * sstride (q < nseq), ping-ponging with b.  Stage s of radix R
// maps a[i + j n/R] (j < R, i < n/R, k = i mod p) through the twiddle
// w^{j k n/(pR)}, a length-R DFT, and stores to b[(i - k) R + k + j p];
// p is the product of the radices of the stages before s.  The output is in
// natural order.  Twiddles come from a table tw[t] = exp(-2 pi i t / n)
// (conjugated for the inverse); the transform is unnormalised.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by SIGN * i
template <typename T, int SIGN>
__device__ __forceinline__ cpx<T> mul_si(cpx<T> a) {
  return SIGN > 0 ? cpx<T>{-a.y, a.x} : cpx<T>{a.y, -a.x};
}

struct FftDesc {
  int32_t n;
  int32_t nst;
  int32_t radix[12];
};

// Radix plan for n = 4^a 3^b 2^c (radix-4 stages first).
static inline bool fft_make_desc(int n, FftDesc* d) {
  d->n = n;
  d->nst = 0;
  int m = n;
  while (m % 4 == 0) { d->radix[d->nst++] = 4; m /= 4; }
  while (m % 3 == 0) { d->radix[d->nst++] = 3; m /= 3; }
  while (m % 2 == 0) { d->radix[d->nst++] = 2; m /= 2; }
  if (m != 1 || d->nst > 12) return false;
  return true;
}

// SIGN = -1: forward (e^{-i...}); SIGN = +1: inverse (unnormalised).
// Returns the buffer holding the result (a or b).  Ends with a barrier.
template <typename T, int SIGN>
__device__ cpx<T>* fft_stockham(cpx<T>* a, cpx<T>* b, int nseq, int sstride, const FftDesc& d,
                                const cpx<T>* __restrict__ tw) {
  const int n = d.n;
  int p = 1;
  for (int s = 0; s < d.nst; ++s) {
    const int R = d.radix[s];
    const int nb = n / R;
    const int total = nseq * nb;
    const int tstride = n / (p * R);
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      const int q = t / nb;
      const int i = t - q * nb;
      const int k = i % p;
      const cpx<T>* src = a + q * sstride;
      cpx<T>* dst = b + q * sstride;
      const int obase = (i - k) * R + k;
      if (R == 4) {
        cpx<T> u0 = src[i], u1 = src[i + nb], u2 = src[i + 2 * nb], u3 = src[i + 3 * nb];
        if (k) {
          cpx<T> w1 = tw[k * tstride], w2 = tw[2 * k * tstride], w3 = tw[3 * k * tstride];
          if (SIGN > 0) { w1 = cconj(w1); w2 = cconj(w2); w3 = cconj(w3); }
          u1 = cmul(u1, w1); u2 = cmul(u2, w2); u3 = cmul(u3, w3);
        }
        cpx<T> s02 = cadd(u0, u2), d02 = csub(u0, u2);
        cpx<T> s13 = cadd(u1, u3), d13 = mul_si<T, SIGN>(csub(u1, u3));
        dst[obase] = cadd(s02, s13);
        dst[obase + p] = cadd(d02, d13);
        dst[obase + 2 * p] = csub(s02, s13);
        dst[obase + 3 * p] = csub(d02, d13);
      } else if (R == 3) {
        cpx<T> u0 = src[i], u1 = src[i + nb], u2 = src[i + 2 * nb];
        if (k) {
          cpx<T> w1 = tw[k * tstride], w2 = tw[2 * k * tstride];
          if (SIGN > 0) { w1 = cconj(w1); w2 = cconj(w2); }
          u1 = cmul(u1, w1); u2 = cmul(u2, w2);
        }
        const T h = (T)0.86602540378443864676;  // sin(2 pi / 3)
        cpx<T> sm = cadd(u1, u2);
        cpx<T> df = cscale(mul_si<T, SIGN>(csub(u1, u2)), h);
        cpx<T> base = {u0.x - (T)0.5 * sm.x, u0.y - (T)0.5 * sm.y};
        dst[obase] = cadd(u0, sm);
        dst[obase + p] = cadd(base, df);
        dst[obase + 2 * p] = csub(base, df);
      } else {
        cpx<T> u0 = src[i], u1 = src[i + nb];
        if (k) {
          cpx<T> w1 = tw[k * tstride];
          if (SIGN > 0) w1 = cconj(w1);
          u1 = cmul(u1, w1);
        }
        dst[obase] = cadd(u0, u1);
        dst[obase + p] = csub(u0, u1);
      }
    }
    __syncthreads();
    cpx<T>* tmp = a;
    a = b;
    b = tmp;
    p *= R;
  }
  return a;
}
