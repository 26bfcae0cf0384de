// Size-specialised row and column kernels of the reduced iteration.  Same
// data layout and results as the generic kernels in solve_kernels.h; the
// transforms are compile-time Stockham passes (fft_reg.h) on one in-place,
// bank-padded LDS buffer, and the pointwise constitutive step runs in
// registers between the last inverse pass and the first forward pass.
#pragma once

#include "fft_reg.h"
#include "solve_kernels.h"

namespace mor_k {

using fftr::Dft;
using fftr::pad16;
using fftr::RList;

// Row kernel configuration for a half length NH (row length L = 2 NH):
// inverse passes RA..., then the register pass RL; forward RL, then RA
// reversed.  RB rows per workgroup, NH/RL threads per row.  The LDS buffer
// holds one strain component of the row block at a time (the register pass
// keeps all C components of a thread's points in registers), so the LDS
// footprint per row is one sequence and many rows fit a CU.  Each (C, NH) has
// RowVar<C, NH>::count variants V (different factorisations and row blocks,
// same results up to FP32 rounding); the host picks one per size (a fixed
// default, or the autotuner's measurement).
template <int C, int NH, int V>
struct RowCfg;
template <int C, int NH>
struct RowVar {
  static constexpr int count = 1;
};
template <> struct RowCfg<3, 32, 0>  { static constexpr int RL = 4, RB = 16; using RA = RList<8>; };
template <> struct RowCfg<3, 32, 1>  { static constexpr int RL = 8, RB = 32; using RA = RList<4>; };
template <> struct RowCfg<3, 32, 2>  { static constexpr int RL = 4, RB = 32; using RA = RList<8>; };
template <> struct RowVar<3, 32> { static constexpr int count = 3; };
template <> struct RowCfg<3, 64, 0>  { static constexpr int RL = 8, RB = 16; using RA = RList<8>; };
template <> struct RowCfg<3, 64, 1>  { static constexpr int RL = 8, RB = 8;  using RA = RList<8>; };
template <> struct RowCfg<3, 64, 2>  { static constexpr int RL = 8, RB = 32; using RA = RList<8>; };
template <> struct RowCfg<3, 64, 3>  { static constexpr int RL = 4, RB = 16; using RA = RList<4, 4>; };
template <> struct RowCfg<3, 64, 4>  { static constexpr int RL = 4, RB = 8;  using RA = RList<4, 4>; };
template <> struct RowCfg<3, 64, 5>  { static constexpr int RL = 8, RB = 16, PS = 5; using RA = RList<8>; };
template <> struct RowVar<3, 64> { static constexpr int count = 6; };
template <> struct RowCfg<3, 128, 0> { static constexpr int RL = 8, RB = 16; using RA = RList<16>; };
template <> struct RowCfg<3, 128, 1> { static constexpr int RL = 8, RB = 8;  using RA = RList<16>; };
template <> struct RowCfg<3, 128, 2> { static constexpr int RL = 8, RB = 32; using RA = RList<16>; };
template <> struct RowCfg<3, 128, 3> { static constexpr int RL = 8, RB = 16; using RA = RList<4, 4>; };
template <> struct RowCfg<3, 128, 4> { static constexpr int RL = 4, RB = 8;  using RA = RList<8, 4>; };
template <> struct RowCfg<3, 128, 5> { static constexpr int RL = 8, RB = 4;  using RA = RList<16>; };
template <> struct RowCfg<3, 128, 6> { static constexpr int RL = 8, RB = 16, PS = 5; using RA = RList<16>; };
template <> struct RowVar<3, 128> { static constexpr int count = 7; };
template <> struct RowCfg<3, 192, 0> { static constexpr int RL = 12, RB = 16; using RA = RList<16>; };
template <> struct RowCfg<3, 192, 1> { static constexpr int RL = 8, RB = 8;  using RA = RList<8, 3>; };
template <> struct RowCfg<3, 192, 2> { static constexpr int RL = 4, RB = 8;  using RA = RList<4, 4, 3>; };
template <> struct RowCfg<3, 192, 3> { static constexpr int RL = 4, RB = 8;  using RA = RList<3, 4, 4>; };
template <> struct RowCfg<3, 192, 4> { static constexpr int RL = 8, RB = 16; using RA = RList<8, 3>; };
template <> struct RowCfg<3, 192, 5> { static constexpr int RL = 4, RB = 16; using RA = RList<4, 4, 3>; };
template <> struct RowCfg<3, 192, 6> { static constexpr int RL = 6, RB = 8;  using RA = RList<4, 8>; };
template <> struct RowCfg<3, 192, 7> { static constexpr int RL = 6, RB = 32; using RA = RList<8, 4>; };
template <> struct RowCfg<3, 192, 8> { static constexpr int RL = 6, RB = 8;  using RA = RList<8, 4>; };
template <> struct RowCfg<3, 192, 9> { static constexpr int RL = 6, RB = 16; using RA = RList<8, 4>; };
template <> struct RowCfg<3, 192, 10> { static constexpr int RL = 12, RB = 8; using RA = RList<16>; };
template <> struct RowVar<3, 192> { static constexpr int count = 11; };
template <> struct RowCfg<3, 256, 0> { static constexpr int RL = 16, RB = 16; using RA = RList<16>; };
template <> struct RowCfg<3, 256, 1> { static constexpr int RL = 8, RB = 8;  using RA = RList<16, 2>; };
template <> struct RowCfg<3, 256, 2> { static constexpr int RL = 8, RB = 16; using RA = RList<4, 8>; };
template <> struct RowCfg<3, 256, 3> { static constexpr int RL = 8, RB = 4;  using RA = RList<4, 8>; };
template <> struct RowCfg<3, 256, 4> { static constexpr int RL = 4, RB = 8;  using RA = RList<8, 8>; };
template <> struct RowCfg<3, 256, 5> { static constexpr int RL = 8, RB = 8;  using RA = RList<4, 8>; };
template <> struct RowVar<3, 256> { static constexpr int count = 6; };
template <> struct RowCfg<6, 32, 0>  { static constexpr int RL = 4, RB = 16; using RA = RList<8>; };
template <> struct RowCfg<6, 32, 1>  { static constexpr int RL = 8, RB = 16; using RA = RList<4>; };
template <> struct RowVar<6, 32> { static constexpr int count = 2; };
template <> struct RowCfg<6, 64, 0>  { static constexpr int RL = 4, RB = 16; using RA = RList<4, 4>; };
template <> struct RowCfg<6, 64, 1>  { static constexpr int RL = 8, RB = 8;  using RA = RList<8>; };
template <> struct RowCfg<6, 64, 2>  { static constexpr int RL = 4, RB = 8;  using RA = RList<4, 4>; };
template <> struct RowVar<6, 64> { static constexpr int count = 3; };
template <> struct RowCfg<6, 128, 0> { static constexpr int RL = 4, RB = 4;  using RA = RList<8, 4>; };
template <> struct RowCfg<6, 128, 1> { static constexpr int RL = 8, RB = 8;  using RA = RList<16>; };
template <> struct RowCfg<6, 128, 2> { static constexpr int RL = 4, RB = 8;  using RA = RList<8, 4>; };
template <> struct RowVar<6, 128> { static constexpr int count = 3; };

// Data padding of a variant: one slot after every 2^PS elements (default 4).
template <typename Cfg, typename = void>
struct PadOf {
  static constexpr int v = 4;
};
template <typename Cfg>
struct PadOf<Cfg, decltype((void)Cfg::PS)> {
  static constexpr int v = Cfg::PS;
};

// Minimum waves per SIMD a variant asks the register allocator for (1: no
// constraint; set where it fits the registers without spills and measured
// faster).
template <typename Cfg, typename = void>
struct WavesOf {
  static constexpr int v = 1;
};
template <typename Cfg>
struct WavesOf<Cfg, decltype((void)Cfg::W)> {
  static constexpr int v = Cfg::W;
};

template <int C, int NH, int V>
constexpr int row_threads() {
  return RowCfg<C, NH, V>::RB * (NH / RowCfg<C, NH, V>::RL);
}
template <int NH, int PS = 4>
constexpr int row_ss() {
  // NH + 1 spectrum slots (Nyquist included); odd, so sequences start on
  // different banks
  return (fftr::padp<PS>(NH) + 1) | 1;
}
template <int NH>
constexpr int row_tw_len() {
  return pad16(2 * NH - 1) + 1;  // padded table of exp(-2 pi i t / (2 NH))
}
template <int C, int NH, int V>
constexpr size_t row_lds_bytes() {
  return (size_t)(row_tw_len<NH>() + RowCfg<C, NH, V>::RB * row_ss<NH, PadOf<RowCfg<C, NH, V>>::v>()) *
         sizeof(cpx<float>);
}

// Raw buffer access to one strain component of an RVE (wave-uniform base,
// byte size below 2^31).  A buffer load whose offset lies at or beyond the
// resource's size is range-checked by the hardware: it touches no memory and
// returns zero.  kOutOfRange is such an offset for every resource built here.
constexpr uint32_t kOutOfRange = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t comp_rsrc(const cpx<float>* base, uint32_t bytes) {
  // stride 0 (raw buffer); the fourth word selects 32-bit data for the gfx9 family
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<cpx<float>*>(base), (short)0, (int)bytes, 0x00020000);
}
typedef int i32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cpx<float> load_or_zero(__amdgpu_buffer_rsrc_t rs, uint32_t byte_off) {
  const i32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)byte_off, 0, 0);
  return {__int_as_float(v.x), __int_as_float(v.y)};
}
__device__ __forceinline__ void store_c(__amdgpu_buffer_rsrc_t rs, uint32_t byte_off, cpx<float> a) {
  i32x2 v;
  v.x = __float_as_int(a.x);
  v.y = __float_as_int(a.y);
  __builtin_amdgcn_raw_buffer_store_b64(v, rs, (int)byte_off, 0, 0);
}

// threadIdx.x, re-read per work item of a persistent loop behind an empty asm
// statement, so that thread-index arithmetic is not hoisted out of the loop
// (hoisting keeps it live across the whole item and doubles the registers).
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// One row block (tile) of one RVE: the work of one workgroup.
template <int C, int NH, int V, int MODE, int MAT>
__device__ __forceinline__ void row_tile(const PlanDev* __restrict__ plans, const int b, const int tile,
                                         RveState* __restrict__ st, cpx<float>* __restrict__ Yl, const Offs& off,
                                         const MatDev& mat, float* __restrict__ jstate, float* __restrict__ out_eps,
                                         float* __restrict__ out_sig, double* __restrict__ sig_part, const int tid) {
  using Cfg = RowCfg<C, NH, V>;
  constexpr int RL = Cfg::RL, RB = Cfg::RB;
  constexpr int PS = PadOf<Cfg>::v;
  constexpr int TR = NH / RL;  // threads per row in the register pass
  constexpr int NT = RB * TR;
  constexpr int SS = row_ss<NH, PS>();
  constexpr int S = Comp<C>::S;
  constexpr int NST = Comp<C>::NST;
  constexpr int L = 2 * NH;
  constexpr int KH = NH / 2 + 1;
  static_assert(NT % 64 == 0, "workgroups are whole wavefronts");
  static_assert(NT % RB == 0, "row block divides the workgroup");
  __builtin_assume(tid >= 0 && tid < NT);  // the launch has NT threads
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  __shared__ int lk[NH + 1];    // last-axis frequency of spectrum entry j
  __shared__ uint32_t kofs[NH + 1];  // byte offset j * rows * 8 of the entry j of last-axis frequency k,
                                    // kOutOfRange if k is not sampled
  if (MODE == MODE_ITER && !st[b].active) return;
  const PlanDev& P = plans[st[b].plan];
  const int rows = P.rows;
  const int r0 = tile * RB;
  if (r0 >= rows) return;
  const int nr = min(RB, rows - r0);
  // T[t] = exp(-2 pi i t / L): the real-FFT twiddles are T[k], the length-NH
  // FFT twiddles are T[2 e].
  cpx<float>* T = reinterpret_cast<cpx<float>*>(smem_raw);
  cpx<float>* buf = T + row_tw_len<NH>();  // RB sequences, one component
  const int nlast = P.nlast;
  for (int t = tid; t < L; t += NT) T[pad16(t)] = P.rtw[t];
  for (int t = tid; t <= NH; t += NT) kofs[t] = kOutOfRange;
  for (int t = tid; t < nlast; t += NT) lk[t] = P.last_k[t];
  __syncthreads();
  // one component spans nlast * rows * 8 < 2^31 bytes for every grid this
  // kernel is built for (nlast <= NH + 1 <= 257 with rows <= 1024 in 2D,
  // nlast <= 129 with rows <= 1024^2 in 3D)
  for (int t = tid; t < nlast; t += NT) kofs[lk[t]] = (uint32_t)t * (uint32_t)rows * 8u;
  __syncthreads();
  cpx<float>* Y = Yl + off.yl[b];
  const int64_t cstride = (int64_t)nlast * rows;
  constexpr int QS = NT / RB;
  const int rg = tid % RB;      // row of this thread in gather / scatter loops
  const bool rlive = rg < nr;
  const int r = tid / TR, i = tid % TR;  // row and butterfly in the register pass
  cpx<float> v[C][RL];

  // ---- inverse transform, one component at a time
  // Gather of the half spectra X[0..NH] of a component: item (k, row) for
  // k = 0..NH/2 loads X[k] and X[NH-k] (zero outside the pattern); rows are the
  // fastest index, so a wavefront reads runs of RB consecutive entries.  The
  // loads of component c+1 are issued before the LDS passes of component c,
  // so their latency overlaps the transform.
  constexpr int GT = KH * RB;             // gather items per component
  constexpr int GU = (GT + NT - 1) / NT;  // items per thread
  cpx<float> xa[GU], xb[GU];
  // Unsampled frequencies read zero through the buffer range check, so the
  // gather has no branches.  Rows past the end of the RVE (rg >= nr) read
  // entries of the next frequency or zero; their results are never stored.
  const uint32_t rowb = (uint32_t)(r0 + rg) * 8u;
  const uint32_t cbytes = (uint32_t)cstride * 8u;
  auto gather = [&](int c) {
    const __amdgpu_buffer_rsrc_t rs = comp_rsrc(Y + (int64_t)c * cstride, cbytes);
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int t = tid + u * NT;  // t % RB == rg
      if (u < GT / NT || t < GT) {  // only the last, partial round checks
        const int k = t / RB;
        xa[u] = load_or_zero(rs, kofs[k] + rowb);
        xb[u] = load_or_zero(rs, kofs[NH - k] + rowb);
      }
    }
  };
  // register-pass twiddles (the same for every component; conjugated for the
  // forward transform)
  cpx<float> rtw[RL];
#pragma unroll
  for (int j = 0; j < RL; ++j) rtw[j] = fftr::twid<+1, 2>(T, j * i * (NH / (TR * RL)));
  gather(0);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    // pack into the length-NH sequence
    //   z[k] = (X[k] + conj X[NH-k]) + i (X[k] - conj X[NH-k]) conj(T[k]);
    // item (k, row) writes z[k] and z[NH-k]; every z position is written.
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int t = tid + u * NT;
      if (u < GT / NT || t < GT) {
        const int k = t / RB;
        cpx<float>* x = buf + rg * SS;
        const cpx<float> Xk = xa[u], Xm = xb[u];
        const cpx<float> a = cadd(Xk, cconj(Xm));
        const cpx<float> d = cmul(csub(Xk, cconj(Xm)), cconj(T[pad16(k)]));
        x[fftr::padp<PS>(k)] = {a.x - d.y, a.y + d.x};
        if (k != 0 && 2 * k != NH) x[fftr::padp<PS>(NH - k)] = {a.x + d.y, d.x - a.y};
      }
    }
    if (c + 1 < C) gather(c + 1);
    __syncthreads();
    fftr::lds_passes<NH, +1, 1, RB, SS, NT, 2, PS, true>(buf, T, tid, typename Cfg::RA{});
    // register pass: last inverse stage (radix RL, span TR)
    {
      const cpx<float>* src = buf + r * SS;
#pragma unroll
      for (int j = 0; j < RL; ++j) v[c][j] = src[fftr::padp<PS>(i + j * TR)];
#pragma unroll
      for (int j = 1; j < RL; ++j) v[c][j] = cmul(v[c][j], rtw[j]);
      Dft<RL, +1>::run(v[c]);
    }
    __syncthreads();
  }

  // ---- pointwise step a): thread holds points 2t, 2t+1 of row r0+r for t = i + j TR
  const bool live = r < nr;
  const int64_t row = r0 + r;
  double acc[S];
#pragma unroll
  for (int s = 0; s < S; ++s) acc[s] = 0.0;
  if (live) {
    const uint8_t* grow = P.g + row * L;
#pragma unroll
    for (int j = 0; j < RL; ++j) {
      const int tt = i + j * TR;
      const int64_t p0 = row * L + 2 * tt;
      const uchar2 gg = *reinterpret_cast<const uchar2*>(grow + 2 * tt);
      float e0[C], e1[C], t0[C], t1[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        e0[c] = v[c][j].x;
        e1[c] = v[c][j].y;
      }
      float sin0[NST], sin1[NST];
      if (MAT == MAT_J2) {
        const float* sp = jstate + off.field[b] * NST;
#pragma unroll
        for (int q = 0; q < NST; ++q) {
          const float2 w = *reinterpret_cast<const float2*>(sp + (int64_t)q * P.N + p0);
          sin0[q] = w.x;
          sin1[q] = w.y;
        }
      }
      if (MODE == MODE_ITER) {
        constitutive<C, MAT>(e0, gg.x, mat, sin0, t0, nullptr, nullptr);
        constitutive<C, MAT>(e1, gg.y, mat, sin1, t1, nullptr, nullptr);
#pragma unroll
        for (int c = 0; c < C; ++c) v[c][j] = {t0[c], t1[c]};
      } else {
        float s0[S], s1[S], so0[NST], so1[NST];
        constitutive<C, MAT>(e0, gg.x, mat, sin0, t0, s0, so0);
        constitutive<C, MAT>(e1, gg.y, mat, sin1, t1, s1, so1);
        if (MAT == MAT_J2) {
          float* sp = jstate + off.field[b] * NST;
#pragma unroll
          for (int q = 0; q < NST; ++q)
            *reinterpret_cast<float2*>(sp + (int64_t)q * P.N + p0) = make_float2(so0[q], so1[q]);
        }
        if (out_eps) {
          float* fe = out_eps + off.field[b] * C;
#pragma unroll
          for (int c = 0; c < C; ++c) *reinterpret_cast<float2*>(fe + (int64_t)c * P.N + p0) = make_float2(e0[c], e1[c]);
        }
        if (out_sig) {
          float* fs = out_sig + off.field[b] * S;
#pragma unroll
          for (int s = 0; s < S; ++s) *reinterpret_cast<float2*>(fs + (int64_t)s * P.N + p0) = make_float2(s0[s], s1[s]);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] += (double)s0[s] + (double)s1[s];
      }
    }
  }
  if (MODE == MODE_FINAL) {
    // all S sums at once (each in the fixed order of a wavefront tree, then
    // the wavefronts in order), with one exchange through LDS
    __shared__ double red[(NT / 64) * S];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
      for (int s = 0; s < S; ++s) acc[s] += __shfl_down(acc[s], o, 64);
    }
    __syncthreads();
    if ((tid & 63) == 0) {
#pragma unroll
      for (int s = 0; s < S; ++s) red[(tid >> 6) * S + s] = acc[s];
    }
    __syncthreads();
    if (tid < S) {
      double w = 0.0;
      for (int q = 0; q < NT / 64; ++q) w += red[q * S + tid];
      sig_part[(off.part[b] + tile) * S + tid] = w;
    }
    return;
  }

  // ---- forward transform, one component at a time
#pragma unroll
  for (int c = 0; c < C; ++c) {
    // register pass: first forward stage (radix RL, span 1)
    Dft<RL, -1>::run(v[c]);
    // With one LDS pass (radix R2 = NH / RL, span RL), output j of this
    // thread lands at input j2 = i of that pass's butterfly k = j, whose
    // twiddle w^{i j} (w = exp(-2 pi i / NH)) is the conjugate of the inverse
    // register pass's rtw[j]: apply it here from registers and run the LDS
    // pass without twiddles.
    constexpr int R2 = fftr::Single<typename Cfg::RA>::v;
    constexpr bool kPreTwiddle = R2 * RL == NH;
    if constexpr (kPreTwiddle) {
#pragma unroll
      for (int j = 1; j < RL; ++j) v[c][j] = cmul(v[c][j], cconj(rtw[j]));
    }
    {
      cpx<float>* dst = buf + r * SS;
#pragma unroll
      for (int j = 0; j < RL; ++j) dst[fftr::padp<PS>(i * RL + j)] = v[c][j];
    }
    __syncthreads();
    if constexpr (kPreTwiddle) {
      fftr::lds_pass<NH, R2, RL, -1, RB, SS, NT, 2, PS, false, true>(buf, T, tid);
    } else {
      fftr::lds_passes<NH, -1, RL, RB, SS, NT, 2, PS, true>(buf, T, tid,
                                                        typename fftr::Rev<typename Cfg::RA, RList<>>::type{});
    }
    // unpack X[k] = (Z[k] + conj Z[NH-k]) / 2 - i T[k] (Z[k] - conj Z[NH-k]) / 2
    // at the sampled frequencies and store them
    if (rlive) {
      const cpx<float>* z = buf + rg * SS;
      const __amdgpu_buffer_rsrc_t rs = comp_rsrc(Y + (int64_t)c * cstride, cbytes);
      for (int j = tid / RB; j < nlast; j += QS) {
        const int k = lk[j];
        const cpx<float> Zk = z[fftr::padp<PS>(k == NH ? 0 : k)];
        const cpx<float> Zc = cconj(z[fftr::padp<PS>(k == 0 ? 0 : NH - k)]);
        const cpx<float> sm = cadd(Zk, Zc);
        const cpx<float> wd = cmul(T[pad16(k)], csub(Zk, Zc));
        store_c(rs, (uint32_t)j * (uint32_t)rows * 8u + rowb, {0.5f * (sm.x + wd.y), 0.5f * (sm.y - wd.x)});
      }
    }
    if (c + 1 < C) __syncthreads();
  }
}

// Grid schedule: workgroup (tile, list position).
template <int C, int NH, int V, int MODE, int MAT>
__global__ __launch_bounds__((row_threads<C, NH, V>())) __attribute__((amdgpu_waves_per_eu(
    MAT == MAT_HOOKE ? WavesOf<RowCfg<C, NH, V>>::v : 1))) void k_row_fast(
    const PlanDev* __restrict__ plans, const int* __restrict__ rve_list, RveState* __restrict__ st,
    cpx<float>* __restrict__ Yl, Offs off, MatDev mat, float* __restrict__ jstate, float* __restrict__ out_eps,
    float* __restrict__ out_sig, double* __restrict__ sig_part) {
  row_tile<C, NH, V, MODE, MAT>(plans, rve_list[blockIdx.y], blockIdx.x, st, Yl, off, mat, jstate, out_eps, out_sig,
                                sig_part, threadIdx.x);
}

// Persistent schedule: a fixed grid walks the (active RVE, tile) items of
// the current iteration; item q is tile q % ntiles of RVE alist[q / ntiles].
// Every workgroup leaves the loop once the items are exhausted.
template <int C, int NH, int V, int MAT>
__global__ __launch_bounds__((row_threads<C, NH, V>())) void k_row_persist(
    const PlanDev* __restrict__ plans, const int* __restrict__ alist, const int* __restrict__ nact, int ntiles,
    RveState* __restrict__ st, cpx<float>* __restrict__ Yl, Offs off, MatDev mat, float* __restrict__ jstate) {
  const int nitems = *nact * ntiles;
#pragma unroll 1
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const int b = __builtin_amdgcn_readfirstlane(alist[q / ntiles]);
    const int tile = __builtin_amdgcn_readfirstlane(q % ntiles);
    row_tile<C, NH, V, MODE_ITER, MAT>(plans, b, tile, st, Yl, off, mat, jstate, nullptr, nullptr, nullptr,
                                       opaque_tid());
    __syncthreads();  // the next item reuses the LDS buffers
  }
}

// Column kernel configuration for axis-0 length N0: forward RF (register,
// from global), then FA...; inverse FA reversed, then RF (register, to
// global).  CB columns per workgroup, N0/RF threads per sequence.  Variants V
// as for the row kernel (RowVar): same results up to FP32 rounding.
template <int C, int N0, int V>
struct ColCfg;
template <int C, int N0>
struct ColVar {
  static constexpr int count = 1;
};
template <> struct ColCfg<3, 64, 0>  { static constexpr int RF = 8,  CB = 8, W = 8; using FA = RList<8>; };
template <> struct ColCfg<3, 64, 1>  { static constexpr int RF = 4,  CB = 4; using FA = RList<4, 4>; };
template <> struct ColVar<3, 64> { static constexpr int count = 2; };
template <> struct ColCfg<3, 128, 0> { static constexpr int RF = 8,  CB = 4, W = 8; using FA = RList<4, 4>; };
template <> struct ColCfg<3, 128, 1> { static constexpr int RF = 16, CB = 8; using FA = RList<8>; };
template <> struct ColCfg<3, 128, 2> { static constexpr int RF = 4,  CB = 2; using FA = RList<8, 4>; };
template <> struct ColVar<3, 128> { static constexpr int count = 3; };
template <> struct ColCfg<3, 256, 0> { static constexpr int RF = 8,  CB = 2, W = 7; using FA = RList<8, 4>; };
template <> struct ColCfg<3, 256, 1> { static constexpr int RF = 4,  CB = 1; using FA = RList<8, 8>; };
template <> struct ColCfg<3, 256, 2> { static constexpr int RF = 16, CB = 4; using FA = RList<16>; };
template <> struct ColCfg<3, 256, 3> { static constexpr int RF = 8,  CB = 4; using FA = RList<8, 4>; };
template <> struct ColCfg<3, 256, 4> { static constexpr int RF = 8,  CB = 2; using FA = RList<4, 8>; };
template <> struct ColCfg<3, 256, 5> { static constexpr int RF = 16, CB = 8; using FA = RList<16>; };
template <> struct ColCfg<3, 256, 6> { static constexpr int RF = 8,  CB = 2, W = 8; using FA = RList<8, 4>; };
template <> struct ColVar<3, 256> { static constexpr int count = 7; };
template <> struct ColCfg<3, 384, 0> { static constexpr int RF = 6,  CB = 1; using FA = RList<8, 8>; };
template <> struct ColCfg<3, 384, 1> { static constexpr int RF = 6,  CB = 2; using FA = RList<8, 8>; };
template <> struct ColCfg<3, 384, 2> { static constexpr int RF = 8,  CB = 4; using FA = RList<8, 6>; };
template <> struct ColCfg<3, 384, 3> { static constexpr int RF = 16, CB = 8; using FA = RList<8, 3>; };
template <> struct ColCfg<3, 384, 4> { static constexpr int RF = 6,  CB = 4; using FA = RList<8, 8>; };
template <> struct ColVar<3, 384> { static constexpr int count = 5; };
template <> struct ColCfg<3, 512, 0> { static constexpr int RF = 8,  CB = 1; using FA = RList<8, 8>; };
template <> struct ColCfg<3, 512, 1> { static constexpr int RF = 16, CB = 4; using FA = RList<8, 4>; };
template <> struct ColCfg<3, 512, 2> { static constexpr int RF = 8,  CB = 2; using FA = RList<8, 8>; };
template <> struct ColVar<3, 512> { static constexpr int count = 3; };
template <> struct ColCfg<6, 64, 0>  { static constexpr int RF = 8,  CB = 4, W = 6; using FA = RList<8>; };
template <> struct ColCfg<6, 128, 0> { static constexpr int RF = 16, CB = 4; using FA = RList<8>; };
template <> struct ColCfg<6, 128, 1> { static constexpr int RF = 8,  CB = 2; using FA = RList<4, 4>; };
template <> struct ColVar<6, 128> { static constexpr int count = 2; };

template <int C, int N0, int V>
constexpr int col_threads() {
  return ColCfg<C, N0, V>::CB * C * (N0 / ColCfg<C, N0, V>::RF);
}
template <int N0>
constexpr int col_ss() {
  return fftr::seq_stride(N0);
}
template <int C, int N0, int V>
constexpr size_t col_lds_bytes() {
  return (size_t)(pad16(N0 - 1) + 1 + C * ColCfg<C, N0, V>::CB * col_ss<N0>()) * sizeof(cpx<float>);
}

// One block of columns (tile) of one RVE.
template <int C, int N0, int V, int MODE>
__device__ __forceinline__ void col_tile(const PlanDev* __restrict__ plans, const int b, const int tile,
                                         RveState* __restrict__ st, const double* __restrict__ ebar,
                                         cpx<float>* __restrict__ Yc, cpx<float>* __restrict__ coef,
                                         const cpx<float>* __restrict__ warm, const Offs& off,
                                         double* __restrict__ part, const MatDev& mat, const int tid) {
  using Cfg = ColCfg<C, N0, V>;
  constexpr int RF = Cfg::RF, CB = Cfg::CB;
  constexpr int TS = N0 / RF;
  constexpr int NT = CB * C * TS;
  constexpr int NSEQ = C * CB;
  constexpr int SS = col_ss<N0>();
  static_assert(NT % 64 == 0, "workgroups are whole wavefronts");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  __shared__ int coff[CB + 1];
  __shared__ double cwt[CB];  // Parseval weight of each column of the block (1 or 2)
  if (MODE == MODE_ITER && !st[b].active) return;
  const PlanDev& P = plans[st[b].plan];
  const int ncol = P.ncol;
  const int j0 = tile * CB;
  if (j0 >= ncol) return;
  const int ncb = min(CB, ncol - j0);
  cpx<float>* tw = reinterpret_cast<cpx<float>*>(smem_raw);
  // one buffer: the forward result tau^, then (after the Green step has read
  // it) the new coefficients and the inverse transform
  cpx<float>* buf = tw + pad16(N0 - 1) + 1;
  for (int t = tid; t < N0; t += NT) tw[pad16(t)] = P.tw0[t];
  if (tid <= CB) coff[tid] = P.col_off[j0 + min(tid, ncb)];
  if (MODE == MODE_ITER && tid < ncb) {
    const int kl = P.last_k[P.col_last[j0 + tid]];
    cwt[tid] = (kl == 0 || 2 * kl == P.nlen) ? 1.0 : 2.0;
  }
  // prefetch this thread's first pattern entry (its loads overlap the FFT)
  const int ncoef = P.ncoef;
  cpx<float>* co = coef + off.coef[b];
  const int ebeg = P.col_off[j0], eend = P.col_off[j0 + ncb];
  int pk0 = 0;
  uint8_t pfl = 0;
  float pn[3] = {0.f, 0.f, 0.f};
  cpx<float> pold[C];
  if (ebeg + tid < eend) {
    const int e = ebeg + tid;
    pk0 = P.coef_k0[e];
    pfl = P.coef_flag[e];
    pn[0] = P.coef_n[3 * e];
    pn[1] = P.coef_n[3 * e + 1];
    pn[2] = P.coef_n[3 * e + 2];
    if (MODE == MODE_ITER) {
#pragma unroll
      for (int c = 0; c < C; ++c) pold[c] = co[(int64_t)c * ncoef + e];
    }
  }
  cpx<float>* Y = Yc + off.yc[b];
  const int64_t cstride = (int64_t)ncol * N0;
  const int s = tid / TS, i = tid % TS;  // sequence s = c * CB + jj
  const int c_s = s / CB, jj_s = s % CB;
  const bool col_live = jj_s < ncb;
  cpx<float>* yline = Y + c_s * cstride + (int64_t)(j0 + jj_s) * N0;
  if (MODE == MODE_ITER) {
    cpx<float> v[RF];
#pragma unroll
    for (int j = 0; j < RF; ++j) v[j] = col_live ? yline[i + j * TS] : cpx<float>{0.f, 0.f};
    Dft<RF, -1>::run(v);
    cpx<float>* dst = buf + s * SS;
#pragma unroll
    for (int j = 0; j < RF; ++j) dst[pad16(i * RF + j)] = v[j];
    __syncthreads();
    fftr::lds_passes<N0, -1, RF, NSEQ, SS, NT, 1>(buf, tw, tid, typename Cfg::FA{});
  } else {
    __syncthreads();
  }
  // step c): Green operator on the block's pattern entries.  A thread
  // handles at most EPT entries and keeps their new coefficients in
  // registers; once every entry has read tau^, the whole buffer is cleared
  // (unconditional stores) and the entries write their coefficients.
  constexpr int EPT = (CB * N0 + NT - 1) / NT;
  const float invN = P.inv_N;
  double dsum = 0.0;
  int kpos[EPT];
  float kre[EPT][C], kim[EPT][C];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    kpos[u] = -1;
    const int e = ebeg + tid + u * NT;
    if (e >= eend) continue;
    int jj = 0;
    while (jj + 1 < ncb && e >= coff[jj + 1]) ++jj;
    const bool first = u == 0;
    const int k0 = first ? pk0 : P.coef_k0[e];
    const uint8_t fl = first ? pfl : P.coef_flag[e];
    float nr_[C], ni_[C];
    if (fl & COEF_ZERO) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        nr_[c] = (float)((double)P.N * ebar[(int64_t)b * C + c]);
        ni_[c] = 0.f;
      }
    } else if (fl & COEF_DEAD) {
#pragma unroll
      for (int c = 0; c < C; ++c) nr_[c] = ni_[c] = 0.f;
    } else if (MODE == MODE_ITER) {
      float tr_[C], ti_[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const cpx<float> w = buf[(c * CB + jj) * SS + pad16(k0)];
        tr_[c] = w.x;
        ti_[c] = w.y;
      }
      float nv[3];
      if (first) {
        nv[0] = pn[0]; nv[1] = pn[1]; nv[2] = pn[2];
      } else {
        nv[0] = P.coef_n[3 * e]; nv[1] = P.coef_n[3 * e + 1]; nv[2] = P.coef_n[3 * e + 2];
      }
      green<C>(nv, tr_, nr_, mat.g_inv_mu0, mat.g_k);
      green<C>(nv, ti_, ni_, mat.g_inv_mu0, mat.g_k);
    } else {
      if (warm && st[b].warm_ok) {
        float wr[C], wi[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const cpx<float> w = warm[off.coef[b] + (int64_t)c * ncoef + e];
          wr[c] = w.x;
          wi[c] = w.y;
        }
        float nv[3];
        if (first) {
          nv[0] = pn[0]; nv[1] = pn[1]; nv[2] = pn[2];
        } else {
          nv[0] = P.coef_n[3 * e]; nv[1] = P.coef_n[3 * e + 1]; nv[2] = P.coef_n[3 * e + 2];
        }
        project_compatible<C>(nv, wr, nr_, mat);
        project_compatible<C>(nv, wi, ni_, mat);
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) nr_[c] = ni_[c] = 0.f;
      }
    }
    if (MODE == MODE_ITER) {
      const double wcol = cwt[jj];
      double d2 = 0.0;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const cpx<float> old = first ? pold[c] : co[(int64_t)c * ncoef + e];
        const double dr = (double)nr_[c] - (double)old.x, di = (double)ni_[c] - (double)old.y;
        d2 += (double)comp_weight<C>(c) * (dr * dr + di * di);
      }
      dsum += wcol * d2;
    }
    kpos[u] = jj * SS + pad16(k0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      co[(int64_t)c * ncoef + e] = {nr_[c], ni_[c]};
      kre[u][c] = nr_[c] * invN;
      kim[u][c] = ni_[c] * invN;
    }
  }
  __syncthreads();  // every entry has read its tau^
  // clear every position of every sequence (pad slots are never read):
  // thread (s, i) of the transform takes positions i + m TS of its sequence,
  // so the offsets are compile-time strides from one per-thread base
  {
    // thread indices re-derived here rather than kept live across the Green step
    const int t2 = opaque_tid();
    const int s2 = t2 / TS, i2 = t2 % TS;
    cpx<float>* seqb = buf + s2 * SS;
#pragma unroll
    for (int m = 0; m < RF; ++m) seqb[pad16(i2 + m * TS)] = {0.f, 0.f};
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    if (kpos[u] < 0) continue;
#pragma unroll
    for (int c = 0; c < C; ++c) buf[c * CB * SS + kpos[u]] = {kre[u][c], kim[u][c]};
  }
  __syncthreads();
  // step d), axis 0: inverse passes, the last one straight to global memory
  fftr::lds_passes<N0, +1, 1, NSEQ, SS, NT, 1>(buf, tw, tid, typename fftr::Rev<typename Cfg::FA, RList<>>::type{});
  {
    cpx<float> v[RF];
    const cpx<float>* src = buf + s * SS;
#pragma unroll
    for (int j = 0; j < RF; ++j) v[j] = src[pad16(i + j * TS)];
    fftr::pass_twiddle<N0, RF, TS, +1>(v, i, tw);
    Dft<RF, +1>::run(v);
    if (col_live) {
#pragma unroll
      for (int j = 0; j < RF; ++j) yline[i + j * TS] = v[j];
    }
  }
  if (MODE == MODE_ITER) {
    __shared__ double red[16];
    const double tot = block_sum_d(dsum, red);
    if (tid == 0) part[off.part[b] + tile] = tot;
  }
}

template <int C, int N0, int V, int MODE>
__global__ __launch_bounds__((col_threads<C, N0, V>())) __attribute__((amdgpu_waves_per_eu(WavesOf<ColCfg<C, N0, V>>::v))) void k_col_fast(
    const PlanDev* __restrict__ plans, const int* __restrict__ rve_list, RveState* __restrict__ st,
    const double* __restrict__ ebar, cpx<float>* __restrict__ Yc, cpx<float>* __restrict__ coef,
    const cpx<float>* __restrict__ warm, Offs off, double* __restrict__ part, MatDev mat) {
  col_tile<C, N0, V, MODE>(plans, rve_list[blockIdx.y], blockIdx.x, st, ebar, Yc, coef, warm, off, part, mat,
                           threadIdx.x);
}

template <int C, int N0, int V>
__global__ __launch_bounds__((col_threads<C, N0, V>())) void k_col_persist(
    const PlanDev* __restrict__ plans, const int* __restrict__ alist, const int* __restrict__ nact, int ntiles,
    RveState* __restrict__ st, const double* __restrict__ ebar, cpx<float>* __restrict__ Yc,
    cpx<float>* __restrict__ coef, Offs off, double* __restrict__ part, MatDev mat) {
  const int nitems = *nact * ntiles;
#pragma unroll 1
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const int b = __builtin_amdgcn_readfirstlane(alist[q / ntiles]);
    const int tile = __builtin_amdgcn_readfirstlane(q % ntiles);
    col_tile<C, N0, V, MODE_ITER>(plans, b, tile, st, ebar, Yc, coef, nullptr, off, part, mat, opaque_tid());
    __syncthreads();
  }
}

// 3D axis-1 kernels (between the row and the column stages), compile-time
// specialised for n1 = 32 / 64 / 128: per workgroup XB consecutive values of
// x0 of one strain component c for one last-axis frequency j2 of one RVE
// (blockIdx.x = c * ceil(n0 / XB) + x0 block), N1/RF threads per sequence.
// Forward: lines of Yl along x1 -> FFT (first pass from HBM into registers,
// the rest in LDS) -> the group's (k1, j2) columns of Yc.  Inverse: those
// columns -> zero-padded lines -> inverse FFT (last pass from registers to
// HBM) -> Yl.  Columns of Yc run along x0, so XB = 16 makes every column
// access a 128-byte run; the XB lines read or written are adjacent in Yl.
template <int N1>
struct MidCfg;
template <> struct MidCfg<32>  { static constexpr int RF = 8, XB = 16; using FA = RList<4>; };
template <> struct MidCfg<64>  { static constexpr int RF = 8, XB = 16; using FA = RList<8>; };
template <> struct MidCfg<128> { static constexpr int RF = 8, XB = 16; using FA = RList<4, 4>; };

template <int N1>
constexpr int mid_threads() {
  return MidCfg<N1>::XB * (N1 / MidCfg<N1>::RF);
}
template <int N1>
constexpr size_t mid_lds_bytes() {
  return (size_t)(pad16(N1 - 1) + 1 + MidCfg<N1>::XB * fftr::seq_stride(N1)) * sizeof(cpx<float>);
}

template <int C, int N1, int DIR>
__global__ __launch_bounds__((mid_threads<N1>())) void k_mid_fast(
    const PlanDev* __restrict__ plans, const int* __restrict__ rve_list, RveState* __restrict__ st,
    cpx<float>* __restrict__ Yl, cpx<float>* __restrict__ Yc, Offs off, int check_active) {
  using Cfg = MidCfg<N1>;
  constexpr int RF = Cfg::RF, XB = Cfg::XB;
  constexpr int TS = N1 / RF;
  constexpr int NT = mid_threads<N1>();
  constexpr int SS = fftr::seq_stride(N1);
  static_assert(NT % 64 == 0, "workgroups are whole wavefronts");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  const int b = rve_list[blockIdx.z];
  if (check_active && !st[b].active) return;
  const PlanDev& P = plans[st[b].plan];
  const int j2 = blockIdx.y;
  if (j2 >= P.nlast) return;
  const int n0 = P.n0;
  const int nxb = (n0 + XB - 1) / XB;
  const int c = blockIdx.x / nxb;
  if (c >= C) return;
  const int x00 = (blockIdx.x - c * nxb) * XB;
  const int nx = min(XB, n0 - x00);
  cpx<float>* tw = reinterpret_cast<cpx<float>*>(smem_raw);
  cpx<float>* buf = tw + pad16(N1 - 1) + 1;
  for (int t = tid; t < N1; t += NT) tw[pad16(t)] = P.tw1[t];
  const int rows = P.rows, nlast = P.nlast, ncol = P.ncol;
  cpx<float>* L = Yl + off.yl[b] + c * (int64_t)nlast * rows;
  cpx<float>* Cc = Yc + off.yc[b] + c * (int64_t)ncol * n0;
  const int ja = P.last_off[j2], jb = P.last_off[j2 + 1];
  const int ng = jb - ja;
  const int s = tid / TS, i = tid % TS;  // sequence s = x0 - x00
  const bool live = s < nx;
  cpx<float>* line = L + (int64_t)j2 * rows + (int64_t)(x00 + s) * N1;
  if (DIR < 0) {
    cpx<float> v[RF];
#pragma unroll
    for (int j = 0; j < RF; ++j) v[j] = live ? line[i + j * TS] : cpx<float>{0.f, 0.f};
    __syncthreads();  // twiddle table
    Dft<RF, -1>::run(v);
    cpx<float>* dst = buf + s * SS;
#pragma unroll
    for (int j = 0; j < RF; ++j) dst[pad16(i * RF + j)] = v[j];
    __syncthreads();
    fftr::lds_passes<N1, -1, RF, XB, SS, NT, 1>(buf, tw, tid, typename Cfg::FA{});
    for (int t = tid; t < ng * nx; t += NT) {
      const int xi = t % nx;
      const int j = ja + t / nx;
      Cc[(int64_t)j * n0 + x00 + xi] = buf[xi * SS + pad16(P.col_k[j])];
    }
  } else {
    for (int t = tid; t < XB * SS; t += NT) buf[t] = {0.f, 0.f};
    __syncthreads();
    for (int t = tid; t < ng * nx; t += NT) {
      const int xi = t % nx;
      const int j = ja + t / nx;
      buf[xi * SS + pad16(P.col_k[j])] = Cc[(int64_t)j * n0 + x00 + xi];
    }
    __syncthreads();
    fftr::lds_passes<N1, +1, 1, XB, SS, NT, 1>(buf, tw, tid,
                                               typename fftr::Rev<typename Cfg::FA, RList<>>::type{});
    cpx<float> v[RF];
    const cpx<float>* src = buf + s * SS;
#pragma unroll
    for (int j = 0; j < RF; ++j) v[j] = src[pad16(i + j * TS)];
    fftr::pass_twiddle<N1, RF, TS, +1>(v, i, tw);
    Dft<RF, +1>::run(v);
    if (live) {
#pragma unroll
      for (int j = 0; j < RF; ++j) line[i + j * TS] = v[j];
    }
  }
}

// Active list of a group for the persistent schedule: the RVEs of `list`
// (in list order) that are still iterating, and their count.
__global__ __launch_bounds__(1024) void k_active_list(const int* __restrict__ list, int nrv,
                                                      const RveState* __restrict__ st, int* __restrict__ alist,
                                                      int* __restrict__ nact) {
  __shared__ int wsum[16];
  int base = 0;
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
  for (int c0 = 0; c0 < nrv; c0 += 1024) {
    const int i = c0 + threadIdx.x;
    const int b = i < nrv ? list[i] : 0;
    const bool on = i < nrv && st[b].active;
    const unsigned long long bal = __ballot(on);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wid] = __popcll(bal);
    __syncthreads();
    int off = base;
    for (int w = 0; w < wid; ++w) off += wsum[w];
    if (on) alist[off + before] = b;
    int tot = 0;
    for (int w = 0; w < 16; ++w) tot += wsum[w];
    __syncthreads();
    base += tot;
  }
  if (threadIdx.x == 0) *nact = base;
}

}  // namespace mor_k
