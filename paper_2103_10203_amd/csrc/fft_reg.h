// Compile-time specialised FFT building blocks: length-R DFTs in registers
// and in-place Stockham passes over an LDS buffer.
//
// Stockham pass (radix R, span P = product of the radices before it, length
// N): butterfly i < N/R of a sequence reads x[i + j N/R] (j < R), multiplies
// input j by w^{j k N/(P R)} with k = i mod P and w = exp(SIGN 2 pi i / N),
// applies the length-R DFT and stores output j at (i - k) R + k + j P.  A
// pass reads everything into registers, waits at a barrier, then writes in
// place, so one LDS buffer suffices.  The last pass of a transform leaves
// thread i holding outputs i + j N/R; the first pass (P = 1) of the next
// transform with the same radix reads exactly those indices, so pointwise
// work between an inverse and a forward transform needs no LDS round trip.
#pragma once

#include "fft_lds.h"

namespace fftr {

template <int SIGN>
__device__ __forceinline__ cpx<float> mul_i(cpx<float> a) {
  return SIGN > 0 ? cpx<float>{-a.y, a.x} : cpx<float>{a.y, -a.x};
}

// cos and sin of 2 pi k / 16 for k = 0..8
__host__ __device__ constexpr float c16(int k) {
  return k == 0 ? 1.0f : k == 1 ? 0.92387953251128674f : k == 2 ? 0.70710678118654752f
       : k == 3 ? 0.38268343236508977f : k == 4 ? 0.0f : k == 5 ? -0.38268343236508977f
       : k == 6 ? -0.70710678118654752f : k == 7 ? -0.92387953251128674f : -1.0f;
}
__host__ __device__ constexpr float s16(int k) {
  return k == 0 ? 0.0f : k == 1 ? 0.38268343236508977f : k == 2 ? 0.70710678118654752f
       : k == 3 ? 0.92387953251128674f : k == 4 ? 1.0f : k == 5 ? 0.92387953251128674f
       : k == 6 ? 0.70710678118654752f : k == 7 ? 0.38268343236508977f : 0.0f;
}

template <int SIGN, int K>
__device__ __forceinline__ cpx<float> rot16(cpx<float> a) {
  // a * exp(SIGN 2 pi i K / 16), K in [0, 8)
  if constexpr (K == 0) return a;
  else if constexpr (K == 4) return mul_i<SIGN>(a);
  else {
    constexpr float c = c16(K);
    constexpr float s = SIGN * s16(K);
    return {a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

template <int R, int SIGN>
struct Dft;

template <int SIGN>
struct Dft<2, SIGN> {
  __device__ __forceinline__ static void run(cpx<float>* v) {
    cpx<float> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int SIGN>
struct Dft<3, SIGN> {
  __device__ __forceinline__ static void run(cpx<float>* v) {
    const float h = 0.86602540378443864676f;
    cpx<float> u0 = v[0], u1 = v[1], u2 = v[2];
    cpx<float> sm = cadd(u1, u2);
    cpx<float> df = cscale(mul_i<SIGN>(csub(u1, u2)), h);
    cpx<float> base = {u0.x - 0.5f * sm.x, u0.y - 0.5f * sm.y};
    v[0] = cadd(u0, sm);
    v[1] = cadd(base, df);
    v[2] = csub(base, df);
  }
};

template <int SIGN>
struct Dft<4, SIGN> {
  __device__ __forceinline__ static void run(cpx<float>* v) {
    cpx<float> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    cpx<float> s13 = cadd(v[1], v[3]), d13 = mul_i<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[1] = cadd(d02, d13);
    v[2] = csub(s02, s13);
    v[3] = csub(d02, d13);
  }
};

template <int SIGN>
struct Dft<6, SIGN> {
  // two length-3 DFTs of the even and odd samples, combined with w6^k
  __device__ __forceinline__ static void run(cpx<float>* v) {
    cpx<float> e[3] = {v[0], v[2], v[4]};
    cpx<float> o[3] = {v[1], v[3], v[5]};
    Dft<3, SIGN>::run(e);
    Dft<3, SIGN>::run(o);
    const float h = 0.86602540378443864676f;
    // w6^1 = 1/2 + SIGN i h, w6^2 = -1/2 + SIGN i h
    const cpx<float> o1 = {0.5f * o[1].x - SIGN * h * o[1].y, 0.5f * o[1].y + SIGN * h * o[1].x};
    const cpx<float> o2 = {-0.5f * o[2].x - SIGN * h * o[2].y, -0.5f * o[2].y + SIGN * h * o[2].x};
    v[0] = cadd(e[0], o[0]);
    v[3] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[4] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[5] = csub(e[2], o2);
  }
};

template <int SIGN>
struct Dft<8, SIGN> {
  __device__ __forceinline__ static void run(cpx<float>* v) {
    cpx<float> e[4] = {v[0], v[2], v[4], v[6]};
    cpx<float> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, SIGN>::run(e);
    Dft<4, SIGN>::run(o);
    o[1] = rot16<SIGN, 2>(o[1]);
    o[2] = rot16<SIGN, 4>(o[2]);
    o[3] = rot16<SIGN, 6>(o[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 4] = csub(e[k], o[k]);
    }
  }
};

template <int SIGN>
struct Dft<12, SIGN> {
  // Good-Thomas 3 x 4 (coprime factors, so no twiddles between the stages):
  // length-3 DFTs over n1 of x[(4 n1 + 3 n2) mod 12] for each n2, then
  // length-4 DFTs over n2 for each k1, output k = (4 k1 + 9 k2) mod 12.
  __device__ __forceinline__ static void run(cpx<float>* v) {
    cpx<float> a[4][3];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < 3; ++n1) a[n2][n1] = v[(4 * n1 + 3 * n2) % 12];
      Dft<3, SIGN>::run(a[n2]);
    }
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      cpx<float> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<4, SIGN>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[(4 * k1 + 9 * k2) % 12] = b[k2];
    }
  }
};

template <int SIGN>
struct Dft<16, SIGN> {
  // 4 x 4: length-4 DFTs over n1 of x[4 n1 + n2], twiddles w16^{n2 k1}, then
  // length-4 DFTs over n2; output k1 + 4 k2.  Fewer operations than halving
  // into two length-8 DFTs (two of the nine twiddles are -i or its multiples
  // of pi/4 and no combining stage of 16 complex additions).
  __device__ __forceinline__ static void run(cpx<float>* v) {
    cpx<float> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      a[n2][0] = v[n2];
      a[n2][1] = v[4 + n2];
      a[n2][2] = v[8 + n2];
      a[n2][3] = v[12 + n2];
      Dft<4, SIGN>::run(a[n2]);
    }
    a[1][1] = rot16<SIGN, 1>(a[1][1]);
    a[1][2] = rot16<SIGN, 2>(a[1][2]);
    a[1][3] = rot16<SIGN, 3>(a[1][3]);
    a[2][1] = rot16<SIGN, 2>(a[2][1]);
    a[2][2] = rot16<SIGN, 4>(a[2][2]);
    a[2][3] = rot16<SIGN, 6>(a[2][3]);
    a[3][1] = rot16<SIGN, 3>(a[3][1]);
    a[3][2] = rot16<SIGN, 6>(a[3][2]);
    a[3][3] = rot16<SIGN, 1>(a[3][3]);  // w16^9 = -w16^1: sign folded below
    a[3][3] = {-a[3][3].x, -a[3][3].y};
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cpx<float> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<4, SIGN>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
    }
  }
};

// LDS position of element i of a sequence: one pad slot after every 16
// elements, so that stride-R accesses (R = 2..16, 8-byte elements) of a
// wavefront spread over all banks.
__host__ __device__ constexpr int pad16(int i) { return i + (i >> 4); }

// Data layout with one pad slot after every 2^PS elements (PS = 4: pad16).
template <int PS>
__host__ __device__ constexpr int padp(int i) {
  return i + (i >> PS);
}

// Sequence stride in LDS for `len` logical elements (odd, so that sequences
// start on different banks).
__host__ __device__ constexpr int seq_stride(int len) {
  return (pad16(len - 1) + 1) | 1;
}

// Twiddle w^{e} from a padded LDS table tw[pad16(t)] = exp(-2 pi i t / (N * TWS)),
// read at stride TWS (conjugated for SIGN > 0).
template <int SIGN, int TWS>
__device__ __forceinline__ cpx<float> twid(const cpx<float>* tw, int e) {
  cpx<float> w = tw[pad16(e * TWS)];  // tables are stored padded, like the data
  return SIGN > 0 ? cconj(w) : w;
}

// Apply the pass twiddles to v[1..R-1] for butterfly phase k.
template <int N, int R, int P, int SIGN, int TWS = 1>
__device__ __forceinline__ void pass_twiddle(cpx<float>* v, int k, const cpx<float>* tw) {
  if constexpr (P > 1) {
    constexpr int ST = N / (P * R);
#pragma unroll
    for (int j = 1; j < R; ++j) v[j] = cmul(v[j], twid<SIGN, TWS>(tw, j * k * ST));
  }
}

// One in-place Stockham pass over NS sequences (base + s*SS, positions
// padded by padp<PS>) by NT threads.  TW = false skips the pass twiddles (the
// producer of the pass's input has applied them).  Work item t is butterfly
// i = t % NB of sequence s = t / NB, or with SF (sequence fastest) butterfly
// t / NS of sequence t % NS: neighbouring lanes then take the same butterfly
// of neighbouring sequences, which an odd sequence stride spreads over all
// banks where the butterflies of one sequence would collide.
template <int N, int R, int P, int SIGN, int NS, int SS, int NT, int TWS, int PS = 4, bool TW = true, bool SF = false>
__device__ __forceinline__ void lds_pass(cpx<float>* buf, const cpx<float>* tw, int tid) {
  constexpr int NB = N / R;
  constexpr int TOTAL = NS * NB;
  constexpr int PER = (TOTAL + NT - 1) / NT;
  cpx<float> v[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int t = tid + q * NT;
    if (TOTAL % NT == 0 || t < TOTAL) {
      // (t / NS) % NB == t / NS here; the modulo tells the compiler i < NB
      const int s = SF ? t % NS : t / NB, i = SF ? (t / NS) % NB : t % NB;
      const int k = i % P;
      const cpx<float>* src = buf + s * SS;
#pragma unroll
      for (int j = 0; j < R; ++j) v[q][j] = src[padp<PS>(i + j * NB)];
      if constexpr (TW) pass_twiddle<N, R, P, SIGN, TWS>(v[q], k, tw);
      Dft<R, SIGN>::run(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int t = tid + q * NT;
    if (TOTAL % NT == 0 || t < TOTAL) {
      const int s = SF ? t % NS : t / NB, i = SF ? (t / NS) % NB : t % NB;
      const int k = i % P;
      cpx<float>* dst = buf + s * SS;
      const int o = (i - k) * R + k;
#pragma unroll
      for (int j = 0; j < R; ++j) dst[padp<PS>(o + j * P)] = v[q][j];
    }
  }
  __syncthreads();
}

template <int... Rs>
struct RList {};

// Runs the passes of RList in order starting with span P.
template <int N, int SIGN, int P, int NS, int SS, int NT, int TWS, int PS = 4, bool SF = false>
__device__ __forceinline__ void lds_passes(cpx<float>*, const cpx<float>*, int, RList<>) {}

template <int N, int SIGN, int P, int NS, int SS, int NT, int TWS, int PS = 4, bool SF = false, int R, int... Rest>
__device__ __forceinline__ void lds_passes(cpx<float>* buf, const cpx<float>* tw, int tid, RList<R, Rest...>) {
  lds_pass<N, R, P, SIGN, NS, SS, NT, TWS, PS, true, SF>(buf, tw, tid);
  lds_passes<N, SIGN, P * R, NS, SS, NT, TWS, PS, SF>(buf, tw, tid, RList<Rest...>{});
}

// Single radix of a one-element list (0 otherwise).
template <typename A>
struct Single {
  static constexpr int v = 0;
};
template <int R>
struct Single<RList<R>> {
  static constexpr int v = R;
};

template <int... Rs>
struct Prod;
template <>
struct Prod<> {
  static constexpr int v = 1;
};
template <int R, int... Rest>
struct Prod<R, Rest...> {
  static constexpr int v = R * Prod<Rest...>::v;
};

// Reverse of a radix list.
template <typename A, typename B>
struct Rev;
template <int... Bs>
struct Rev<RList<>, RList<Bs...>> {
  using type = RList<Bs...>;
};
template <int A0, int... As, int... Bs>
struct Rev<RList<A0, As...>, RList<Bs...>> {
  using type = typename Rev<RList<As...>, RList<A0, Bs...>>::type;
};

}  // namespace fftr
