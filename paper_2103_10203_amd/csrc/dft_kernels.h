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
// a_hi b_hi + a_hi b_lo + a_lo b_hi in FP32 with the bf16 MFMA (32x32x8).
//
// Workgroup = 4 wavefronts computing a 64 (m) x 64 (n) output tile, each
// wavefront one 32 x 32 block; K is staged through LDS 32 at a time.
// Requires rows % 64 == 0 and L % 64 == 0 (checked by the host).
#pragma once

#include "solve_kernels.h"

namespace mor_k {

enum { DFT_F32 = 0, DFT_X3 = 1 };

typedef short dft_bf16x4 __attribute__((ext_vector_type(4)));
typedef float dft_f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ unsigned short dft_f2bf(float f) {
  // round to nearest even (finite inputs)
  const unsigned int u = __float_as_uint(f);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float dft_bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

constexpr int DFT_T = 64;   // output tile edge
constexpr int DFT_KC = 32;  // K staged per LDS round
constexpr int DFT_LD = DFT_KC + 4;

// Accumulate the wave's 32x32 block over one staged K chunk.  As[m][k],
// Bs[n][k] (k contiguous).
template <int PREC>
__device__ __forceinline__ void dft_mfma_chunk(const float (*As)[DFT_LD], const float (*Bs)[DFT_LD], int wm, int wn,
                                               int lane, dft_f32x16& acc) {
  const int r = lane % 32;
  if (PREC == DFT_F32) {
    const int kq = lane / 32;
#pragma unroll
    for (int ks = 0; ks < DFT_KC; ks += 2) {
      const float a = As[wm + r][ks + kq];
      const float b = Bs[wn + r][ks + kq];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
  } else {
    const int kq = (lane / 32) * 4;
#pragma unroll
    for (int ks = 0; ks < DFT_KC; ks += 8) {
      const float4 av = *reinterpret_cast<const float4*>(&As[wm + r][ks + kq]);
      const float4 bv = *reinterpret_cast<const float4*>(&Bs[wn + r][ks + kq]);
      const float aa[4] = {av.x, av.y, av.z, av.w};
      const float bb[4] = {bv.x, bv.y, bv.z, bv.w};
      dft_bf16x4 ah, al, bh, bl;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const unsigned short h1 = dft_f2bf(aa[i]);
        const unsigned short h2 = dft_f2bf(bb[i]);
        ah[i] = (short)h1;
        al[i] = (short)dft_f2bf(aa[i] - dft_bf2f(h1));
        bh[i] = (short)h2;
        bl[i] = (short)dft_f2bf(bb[i] - dft_bf2f(h2));
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(al, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, bh, acc, 0, 0, 0);
    }
  }
}

// Shared set-up: twiddle table T[t] = exp(-2 pi i t / L) and the sampled
// last-axis frequencies k_j of the RVE's plan.
__device__ __forceinline__ void dft_tables(const PlanDev& P, cpx<float>* T, int* lk, int L, int nlast) {
  for (int t = threadIdx.x; t < L; t += blockDim.x) T[t] = P.rtw[t];
  for (int t = threadIdx.x; t < nlast; t += blockDim.x) lk[t] = P.last_k[t];
}

// Inverse: Yl (spectra, [C][nlast][rows]) -> E ([C*rows][L] real field).
// grid (L / 64, C rows / 64, RVEs); LMAX >= L.
template <int PREC, int LMAX>
__global__ __launch_bounds__(256) void k_dft_inv(const PlanDev* __restrict__ plans, const int* __restrict__ rve_list,
                                                 const RveState* __restrict__ st, const cpx<float>* __restrict__ Yl,
                                                 Offs off, float* __restrict__ E, int C, int mode_iter) {
  __shared__ float As[DFT_T][DFT_LD];
  __shared__ float Bs[DFT_T][DFT_LD];
  __shared__ cpx<float> T[LMAX];
  __shared__ int lk[LMAX / 2 + 1];
  const int b = rve_list[blockIdx.z];
  if (mode_iter && !st[b].active) return;
  const PlanDev& P = plans[st[b].plan];
  const int rows = P.rows, L = P.nlen, nlast = P.nlast;
  const int n0 = blockIdx.x * DFT_T, m0 = blockIdx.y * DFT_T;
  if (n0 >= L || m0 >= C * rows) return;
  dft_tables(P, T, lk, L, nlast);
  const int c = m0 / rows, row0 = m0 % rows;
  const cpx<float>* Y = Yl + off.yl[b] + (int64_t)c * nlast * rows + row0;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = (wave / 2) * 32, wn = (wave % 2) * 32;
  dft_f32x16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  const int K = 2 * nlast;
  __syncthreads();
  for (int k0 = 0; k0 < K; k0 += DFT_KC) {
    const int j0 = k0 / 2;
    // A: 64 rows x 16 spectrum entries (complex -> two k columns)
    for (int t = tid; t < DFT_T * (DFT_KC / 2); t += 256) {
      const int mm = t % DFT_T, jj = t / DFT_T;
      const int j = j0 + jj;
      cpx<float> v = {0.f, 0.f};
      if (j < nlast) v = Y[(int64_t)j * rows + mm];
      As[mm][2 * jj] = v.x;
      As[mm][2 * jj + 1] = v.y;
    }
    // B: Binv[k][x] for x in the tile
    for (int t = tid; t < DFT_T * (DFT_KC / 2); t += 256) {
      const int nn = t % DFT_T, jj = t / DFT_T;
      const int j = j0 + jj;
      float cr = 0.f, ci = 0.f;
      if (j < nlast) {
        const int k = lk[j];
        const float w = (k == 0 || 2 * k == L) ? 1.f : 2.f;
        const cpx<float> tw = T[(int)(((int64_t)k * (n0 + nn)) % L)];
        cr = w * tw.x;
        ci = w * tw.y;
      }
      Bs[nn][2 * jj] = cr;
      Bs[nn][2 * jj + 1] = ci;
    }
    __syncthreads();
    dft_mfma_chunk<PREC>(As, Bs, wm, wn, lane, acc);
    __syncthreads();
  }
  // D layout: lane -> column n = lane % 32; element i -> row (i/4)*8 + (lane/32)*4 + i%4
  float* Eb = E + off.field[b] * C;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int mm = wm + (i / 4) * 8 + (lane / 32) * 4 + (i % 4);
    const int x = n0 + wn + lane % 32;
    Eb[(int64_t)(m0 + mm) * L + x] = acc[i];
  }
}

// Forward: tau ([C*rows][L]) -> Yl spectra at the sampled frequencies.
// grid (ceil(2 nlast / 64), C rows / 64, RVEs).
template <int PREC, int LMAX>
__global__ __launch_bounds__(256) void k_dft_fwd(const PlanDev* __restrict__ plans, const int* __restrict__ rve_list,
                                                 const RveState* __restrict__ st, cpx<float>* __restrict__ Yl,
                                                 Offs off, const float* __restrict__ E, int C) {
  __shared__ float As[DFT_T][DFT_LD];
  __shared__ float Bs[DFT_T][DFT_LD];
  __shared__ cpx<float> T[LMAX];
  __shared__ int lk[LMAX / 2 + 1];
  __shared__ float Cs[DFT_T][DFT_T + 1];
  const int b = rve_list[blockIdx.z];
  if (!st[b].active) return;
  const PlanDev& P = plans[st[b].plan];
  const int rows = P.rows, L = P.nlen, nlast = P.nlast;
  const int n0 = blockIdx.x * DFT_T, m0 = blockIdx.y * DFT_T;
  if (n0 >= 2 * nlast || m0 >= C * rows) return;
  dft_tables(P, T, lk, L, nlast);
  const int c = m0 / rows, row0 = m0 % rows;
  const float* A = E + off.field[b] * C + (int64_t)m0 * L;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = (wave / 2) * 32, wn = (wave % 2) * 32;
  dft_f32x16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  __syncthreads();
  for (int k0 = 0; k0 < L; k0 += DFT_KC) {
    for (int t = tid; t < DFT_T * DFT_KC; t += 256) {
      const int kk = t % DFT_KC, mm = t / DFT_KC;
      As[mm][kk] = A[(int64_t)mm * L + k0 + kk];
    }
    // B: Bfwd[x][n], n = 2j + p
    for (int t = tid; t < DFT_T * DFT_KC; t += 256) {
      const int kk = t % DFT_KC, nn = t / DFT_KC;
      const int n = n0 + nn, j = n / 2;
      float v = 0.f;
      if (j < nlast) {
        const cpx<float> tw = T[(int)(((int64_t)lk[j] * (k0 + kk)) % L)];
        v = (n & 1) ? tw.y : tw.x;
      }
      Bs[nn][kk] = v;
    }
    __syncthreads();
    dft_mfma_chunk<PREC>(As, Bs, wm, wn, lane, acc);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int mm = wm + (i / 4) * 8 + (lane / 32) * 4 + (i % 4);
    Cs[mm][wn + lane % 32] = acc[i];
  }
  __syncthreads();
  // store complex Y[c][j][row]: rows fastest, 8-byte entries
  cpx<float>* Y = Yl + off.yl[b] + (int64_t)c * nlast * rows + row0;
  for (int t = tid; t < DFT_T * (DFT_T / 2); t += 256) {
    const int mm = t % DFT_T, jj = t / DFT_T;
    const int j = n0 / 2 + jj;
    if (j < nlast) Y[(int64_t)j * rows + mm] = {Cs[mm][2 * jj], Cs[mm][2 * jj + 1]};
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
