// Partial DFT of the last grid axis as dense GEMMs on the matrix cores
// (steps b and d restricted to the sampled last-axis frequencies), the
// alternative to the row kernel's FFT:
//
//   inverse  E[m][x] = sum_j w_j Re(Y[c][j][row] exp(+2 pi i k_j x / L))
//                    = sum_kk A[m][kk] Binv[kk][x],   m = c rows + row,
//            A[m][2j] = Re Y, A[m][2j+1] = Im Y,
//            Binv[2j][x] = w_j cos(theta), Binv[2j+1][x] = -w_j sin(theta),
//            theta = 2 pi (k_j x mod L) / L, w_j = 1 for k_j in {0, L/2}, else 2
//            (the Hermitian extension of the half spectrum);
//   forward  Y[c][j][row] = sum_x tau[m][x] exp(-2 pi i k_j x / L)
//            = F[m][2j] + i F[m][2j+1],  F = tau Bfwd,
//            Bfwd[x][2j] = cos(theta), Bfwd[x][2j+1] = -sin(theta).
//
// Both are unnormalised, like the FFT path they replace.  The twiddle
// operands are generated per tile from a table of exp(-2 pi i t / L) in LDS.
// Precision: PREC_F32 uses the FP32 MFMA (32x32x2); PREC_X3 splits every
// operand a = a_hi + a_lo into two bfloat16 numbers and accumulates
// a_hi b_hi + a_hi b_lo + a_lo b_hi in FP32 with the bf16 MFMA (32x32x16).
//
// Workgroup = 4 wavefronts computing a (64 MB) (m) x 64 (n) output tile,
// each wavefront MB blocks of 32 x 32; K is staged through LDS 32 at a time.
// Requires rows % 64 == 0 and L % 64 == 0 (checked by the host).
#pragma once

#include "solve_kernels.h"

namespace mor_k {

enum { DFT_F32 = 0, DFT_X3 = 1 };

typedef short dft_bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 dft_bf16x8 __attribute__((ext_vector_type(8)));
typedef float dft_f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ unsigned short dft_f2bf(float f) {
  // round to nearest even (finite inputs)
  const unsigned int u = __float_as_uint(f);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float dft_bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

constexpr int DFT_T = 64;   // output tile edge
constexpr int DFT_KC = 32;  // K staged per LDS round
constexpr int DFT_LD = DFT_KC + 4;  // FP32 staging row (floats)
constexpr int DFT_LH = DFT_KC + 8;  // split-bf16 staging row (bf16 values, 16-byte aligned rows)

// Staged operand tiles of one K chunk: FP32 for PREC_F32; for PREC_X3 every
// value is split once, when it is staged, into its bf16 high part and the
// bf16 rounding of the remainder (no conversions in the MFMA loop).
template <int PREC, int MT>
struct DftTiles;
// Values are staged four consecutive k at a time (k a multiple of 4), so
// every LDS store is 16 bytes (FP32) or two of 8 bytes (bf16 high and low).
// MT rows of A (64 or 128), 64 rows of B.
template <int MT>
struct DftTiles<DFT_F32, MT> {
  float A[MT][DFT_LD], B[DFT_T][DFT_LD];
  __device__ __forceinline__ void put_a(int m, int k, float4 v) { *reinterpret_cast<float4*>(&A[m][k]) = v; }
  __device__ __forceinline__ void put_b(int n, int k, float4 v) { *reinterpret_cast<float4*>(&B[n][k]) = v; }
};
template <int MT>
struct DftTiles<DFT_X3, MT> {
  unsigned short Ah[MT][DFT_LH], Al[MT][DFT_LH], Bh[DFT_T][DFT_LH], Bl[DFT_T][DFT_LH];
  __device__ __forceinline__ static void split(float4 v, unsigned short (*H)[DFT_LH], unsigned short (*Lo)[DFT_LH],
                                               int r, int k) {
    const float a[4] = {v.x, v.y, v.z, v.w};
    dft_bf16x4 h, l;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const unsigned short hi = dft_f2bf(a[i]);
      h[i] = (short)hi;
      l[i] = (short)dft_f2bf(a[i] - dft_bf2f(hi));
    }
    *reinterpret_cast<dft_bf16x4*>(&H[r][k]) = h;
    *reinterpret_cast<dft_bf16x4*>(&Lo[r][k]) = l;
  }
  __device__ __forceinline__ void put_a(int m, int k, float4 v) { split(v, Ah, Al, m, k); }
  __device__ __forceinline__ void put_b(int n, int k, float4 v) { split(v, Bh, Bl, n, k); }
};

// Accumulate the wave's MB 32x32 blocks (rows wm + 32 i, columns wn) over
// one staged K chunk (A[m][k], B[n][k], k contiguous): each B fragment read
// serves MB products.
template <int MT, int MB>
__device__ __forceinline__ void dft_mfma_chunk(const DftTiles<DFT_F32, MT>& t, int wm, int wn, int lane,
                                               dft_f32x16 (&acc)[MB]) {
  const int r = lane % 32, kq = lane / 32;
#pragma unroll
  for (int ks = 0; ks < DFT_KC; ks += 2) {
    const float b = t.B[wn + r][ks + kq];
#pragma unroll
    for (int i = 0; i < MB; ++i)
      acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(t.A[wm + 32 * i + r][ks + kq], b, acc[i], 0, 0, 0);
  }
}
// gfx950's 32x32x16 bf16 MFMA: lane l holds row l % 32 and the eight
// consecutive k (l / 32) * 8 .. + 7 of each operand (16-byte LDS reads).
template <int MT, int MB>
__device__ __forceinline__ void dft_mfma_chunk(const DftTiles<DFT_X3, MT>& t, int wm, int wn, int lane,
                                               dft_f32x16 (&acc)[MB]) {
  const int r = lane % 32, kq = (lane / 32) * 8;
#pragma unroll
  for (int ks = 0; ks < DFT_KC; ks += 16) {
    const dft_bf16x8 bh = *reinterpret_cast<const dft_bf16x8*>(&t.Bh[wn + r][ks + kq]);
    const dft_bf16x8 bl = *reinterpret_cast<const dft_bf16x8*>(&t.Bl[wn + r][ks + kq]);
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const dft_bf16x8 ah = *reinterpret_cast<const dft_bf16x8*>(&t.Ah[wm + 32 * i + r][ks + kq]);
      const dft_bf16x8 al = *reinterpret_cast<const dft_bf16x8*>(&t.Al[wm + 32 * i + r][ks + kq]);
      // smallest products first
      acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[i], 0, 0, 0);
      acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[i], 0, 0, 0);
      acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[i], 0, 0, 0);
    }
  }
}

// Shared set-up: twiddle table T[t] = exp(-2 pi i t / L) and the sampled
// last-axis frequencies k_j of the RVE's plan.
__device__ __forceinline__ void dft_tables(const PlanDev& P, cpx<float>* T, int* lk, int L, int nlast) {
  for (int t = threadIdx.x; t < L; t += blockDim.x) T[t] = P.rtw[t];
  for (int t = threadIdx.x; t < nlast; t += blockDim.x) lk[t] = P.last_k[t];
}

// Twiddle index (k x) mod L for k, x < L <= 512 (the product fits 32 bits);
// a mask when L is a power of two (uniform across the launch).
__device__ __forceinline__ int dft_twi(int k, int x, int L) {
  const unsigned p = (unsigned)k * (unsigned)x;
  return (int)((L & (L - 1)) == 0 ? (p & (unsigned)(L - 1)) : p % (unsigned)L);
}

// Inverse: Yl (spectra, [C][nlast][rows]) -> E ([C*rows][L] real field).
// Workgroup tile (64 MB rows) x 64 columns, MB 32x32 blocks per wavefront.
// grid (L / 64, C rows / (64 MB), RVEs); LMAX >= L; rows % (64 MB) == 0.
template <int PREC, int LMAX, int MB>
__global__ __launch_bounds__(256) void k_dft_inv(const PlanDev* __restrict__ plans, const int* __restrict__ rve_list,
                                                 const RveState* __restrict__ st, const cpx<float>* __restrict__ Yl,
                                                 Offs off, float* __restrict__ E, int C, int mode_iter) {
  constexpr int MT = DFT_T * MB;
  __shared__ __attribute__((aligned(16))) DftTiles<PREC, MT> tl;
  __shared__ cpx<float> T[LMAX];
  __shared__ int lk[LMAX / 2 + 1];
  const int b = rve_list[blockIdx.z];
  if (mode_iter && !st[b].active) return;
  const PlanDev& P = plans[st[b].plan];
  const int rows = P.rows, L = P.nlen, nlast = P.nlast;
  const int n0 = blockIdx.x * DFT_T, m0 = blockIdx.y * MT;
  if (n0 >= L || m0 >= C * rows) return;
  dft_tables(P, T, lk, L, nlast);
  const int c = m0 / rows, row0 = m0 % rows;
  const cpx<float>* Y = Yl + off.yl[b] + (int64_t)c * nlast * rows + row0;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = (wave / 2) * 32 * MB, wn = (wave % 2) * 32;
  dft_f32x16 acc[MB];
#pragma unroll
  for (int q = 0; q < MB; ++q)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[q][i] = 0.f;
  const int K = 2 * nlast;
  // A: MT rows x 16 spectrum entries (complex -> two k columns), two
  // entries (four k columns) per item; the next chunk's entries are loaded
  // into registers before this chunk's MFMAs
  constexpr int AI = MT * (DFT_KC / 4) / 256;
  float4 pa[AI];
  auto load_a = [&](int j0) {
#pragma unroll
    for (int q = 0; q < AI; ++q) {
      const int t = tid + q * 256;
      const int mm = t % MT, j = j0 + 2 * (t / MT);
      cpx<float> v0 = {0.f, 0.f}, v1 = {0.f, 0.f};
      if (j < nlast) v0 = Y[(int64_t)j * rows + mm];
      if (j + 1 < nlast) v1 = Y[(int64_t)(j + 1) * rows + mm];
      pa[q] = make_float4(v0.x, v0.y, v1.x, v1.y);
    }
  };
  load_a(0);
  __syncthreads();
  for (int k0 = 0; k0 < K; k0 += DFT_KC) {
    const int j0 = k0 / 2;
#pragma unroll
    for (int q = 0; q < AI; ++q) {
      const int t = tid + q * 256;
      tl.put_a(t % MT, 4 * (t / MT), pa[q]);
    }
    // B: Binv[k][x] for x in the tile
    for (int t = tid; t < DFT_T * (DFT_KC / 4); t += 256) {
      const int nn = t % DFT_T, jg = t / DFT_T;
      float cv[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = j0 + 2 * jg + h;
        if (j < nlast) {
          const int k = lk[j];
          const float w = (k == 0 || 2 * k == L) ? 1.f : 2.f;
          const cpx<float> tw = T[dft_twi(k, n0 + nn, L)];
          cv[2 * h] = w * tw.x;
          cv[2 * h + 1] = w * tw.y;
        }
      }
      tl.put_b(nn, 4 * jg, make_float4(cv[0], cv[1], cv[2], cv[3]));
    }
    __syncthreads();
    if (k0 + DFT_KC < K) load_a(j0 + DFT_KC / 2);
    dft_mfma_chunk<MT, MB>(tl, wm, wn, lane, acc);
    __syncthreads();
  }
  // D layout: lane -> column n = lane % 32; element i -> row (i/4)*8 + (lane/32)*4 + i%4
  float* Eb = E + off.field[b] * C;
#pragma unroll
  for (int q = 0; q < MB; ++q)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int mm = wm + 32 * q + (i / 4) * 8 + (lane / 32) * 4 + (i % 4);
      const int x = n0 + wn + lane % 32;
      Eb[(int64_t)(m0 + mm) * L + x] = acc[q][i];
    }
}

// Forward: tau ([C*rows][L]) -> Yl spectra at the sampled frequencies.
// Workgroup tile (64 MB rows) x 64 columns; grid (ceil(2 nlast / 64),
// C rows / (64 MB), RVEs).
template <int PREC, int LMAX, int MB>
__global__ __launch_bounds__(256) void k_dft_fwd(const PlanDev* __restrict__ plans, const int* __restrict__ rve_list,
                                                 const RveState* __restrict__ st, cpx<float>* __restrict__ Yl,
                                                 Offs off, const float* __restrict__ E, int C) {
  constexpr int MT = DFT_T * MB;
  // the operand tiles and the result tile are never live together
  union Smem {
    DftTiles<PREC, MT> tl;
    float Cs[MT][DFT_T + 1];
  };
  __shared__ __attribute__((aligned(16))) Smem sm;
  DftTiles<PREC, MT>& tl = sm.tl;
  __shared__ cpx<float> T[LMAX];
  __shared__ int lk[LMAX / 2 + 1];
  const int b = rve_list[blockIdx.z];
  if (!st[b].active) return;
  const PlanDev& P = plans[st[b].plan];
  const int rows = P.rows, L = P.nlen, nlast = P.nlast;
  const int n0 = blockIdx.x * DFT_T, m0 = blockIdx.y * MT;
  if (n0 >= 2 * nlast || m0 >= C * rows) return;
  dft_tables(P, T, lk, L, nlast);
  const int c = m0 / rows, row0 = m0 % rows;
  const float* A = E + off.field[b] * C + (int64_t)m0 * L;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = (wave / 2) * 32 * MB, wn = (wave % 2) * 32;
  dft_f32x16 acc[MB];
#pragma unroll
  for (int q = 0; q < MB; ++q)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[q][i] = 0.f;
  // four consecutive x per item (16-byte loads; L and k0 are multiples of 32);
  // the next chunk's items are loaded into registers before this chunk's
  // MFMAs, so their latency overlaps the products
  constexpr int AI = MT * (DFT_KC / 4) / 256;
  float4 pa[AI];
  auto load_a = [&](int k0) {
#pragma unroll
    for (int q = 0; q < AI; ++q) {
      const int t = tid + q * 256;
      const int kq = (t % (DFT_KC / 4)) * 4, mm = t / (DFT_KC / 4);
      pa[q] = *reinterpret_cast<const float4*>(&A[(int64_t)mm * L + k0 + kq]);
    }
  };
  load_a(0);
  __syncthreads();
  for (int k0 = 0; k0 < L; k0 += DFT_KC) {
#pragma unroll
    for (int q = 0; q < AI; ++q) {
      const int t = tid + q * 256;
      tl.put_a(t / (DFT_KC / 4), (t % (DFT_KC / 4)) * 4, pa[q]);
    }
    // B: Bfwd[x][n], n = 2j + p
    for (int t = tid; t < DFT_T * (DFT_KC / 4); t += 256) {
      const int kq = (t % (DFT_KC / 4)) * 4, nn = t / (DFT_KC / 4);
      const int n = n0 + nn, j = n / 2;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (j < nlast) {
        const int k = lk[j];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const cpx<float> tw = T[dft_twi(k, k0 + kq + q, L)];
          v[q] = (n & 1) ? tw.y : tw.x;
        }
      }
      tl.put_b(nn, kq, make_float4(v[0], v[1], v[2], v[3]));
    }
    __syncthreads();
    if (k0 + DFT_KC < L) load_a(k0 + DFT_KC);
    dft_mfma_chunk<MT, MB>(tl, wm, wn, lane, acc);
    __syncthreads();
  }
  // (the loop ended with a barrier: every wave is done with the tiles)
#pragma unroll
  for (int q = 0; q < MB; ++q)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int mm = wm + 32 * q + (i / 4) * 8 + (lane / 32) * 4 + (i % 4);
      sm.Cs[mm][wn + lane % 32] = acc[q][i];
    }
  __syncthreads();
  // store complex Y[c][j][row]: rows fastest, 8-byte entries
  cpx<float>* Y = Yl + off.yl[b] + (int64_t)c * nlast * rows + row0;
  for (int t = tid; t < MT * (DFT_T / 2); t += 256) {
    const int mm = t % MT, jj = t / MT;
    const int j = n0 / 2 + jj;
    if (j < nlast) Y[(int64_t)j * rows + mm] = {sm.Cs[mm][2 * jj], sm.Cs[mm][2 * jj + 1]};
  }
}

// Pointwise step a) between the two GEMMs, on the field E ([C][rows][L] per
// RVE, in place: strain in, polarisation out), and the final evaluation
// (stress sums per row block, field outputs, J2 commit).  grid (ceil(rows /
// RB), RVEs), 256 threads.
template <int C, int MODE, int MAT>
__global__ __launch_bounds__(256) void k_dft_point(const PlanDev* __restrict__ plans, const int* __restrict__ rve_list,
                                                   const RveState* __restrict__ st, Offs off, MatDev mat,
                                                   float* __restrict__ E, float* __restrict__ jstate,
                                                   float* __restrict__ out_eps, float* __restrict__ out_sig,
                                                   double* __restrict__ sig_part, int RB) {
  constexpr int S = Comp<C>::S;
  constexpr int NST = Comp<C>::NST;
  const int b = rve_list[blockIdx.y];
  if (MODE == MODE_ITER && !st[b].active) return;
  const PlanDev& P = plans[st[b].plan];
  const int rows = P.rows, L = P.nlen;
  const int r0 = blockIdx.x * RB;
  if (r0 >= rows) return;
  const int64_t N = P.N;
  const int64_t q0 = (int64_t)r0 * L, q1 = (int64_t)min(rows, r0 + RB) * L;
  float* Eb = E + off.field[b] * C;
  double acc[S];
#pragma unroll
  for (int s = 0; s < S; ++s) acc[s] = 0.0;
  for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
    float e[C], t[C], sin_[NST];
#pragma unroll
    for (int c = 0; c < C; ++c) e[c] = Eb[(int64_t)c * N + q];
    if (MAT == MAT_J2) {
      const float* sp = jstate + off.field[b] * NST;
#pragma unroll
      for (int k = 0; k < NST; ++k) sin_[k] = sp[(int64_t)k * N + q];
    }
    const int ph = P.g[q];
    if (MODE == MODE_ITER) {
      constitutive<C, MAT>(e, ph, mat, sin_, t, nullptr, nullptr);
#pragma unroll
      for (int c = 0; c < C; ++c) Eb[(int64_t)c * N + q] = t[c];
    } else {
      float s[S], so[NST];
      constitutive<C, MAT>(e, ph, mat, sin_, t, s, so);
      if (MAT == MAT_J2) {
        float* sp = jstate + off.field[b] * NST;
#pragma unroll
        for (int k = 0; k < NST; ++k) sp[(int64_t)k * N + q] = so[k];
      }
      if (out_eps) {
#pragma unroll
        for (int c = 0; c < C; ++c) out_eps[off.field[b] * C + (int64_t)c * N + q] = e[c];
      }
      if (out_sig) {
#pragma unroll
        for (int k = 0; k < S; ++k) out_sig[off.field[b] * S + (int64_t)k * N + q] = s[k];
      }
#pragma unroll
      for (int k = 0; k < S; ++k) acc[k] += (double)s[k];
    }
  }
  if (MODE == MODE_FINAL) {
    __shared__ double red[16];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double w = block_sum_d(acc[s], red);
      if (threadIdx.x == 0) sig_part[(off.part[b] + blockIdx.x) * S + s] = w;
    }
  }
}

}  // namespace mor_k
