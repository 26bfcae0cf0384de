// Adapted sampling pattern and plan tables (paper Sec. 4.2; reduced scheme of
// Sec. 4), for one microstructure or a batch of them on one grid, and the
// fixed radial pattern of Sec. 4.1 as the alternative.  Every step runs on
// the device, each as one launch over the batch:
//   1. FP64 FFT of the phase indicator g (Stockham along each axis),
//   2. per-frequency ranking keys and pair representatives (radial pattern:
//      key 1 on the rasterised lines, 0 elsewhere),
//   3. bitonic sort of the conjugate pairs by (key desc, |s|^2, lexrank), and
//      the merge of the self-conjugate frequencies into that order,
//   4. pair-atomic selection of the first M frequencies,
//   5. compaction of the selection mask into sorted linear indices,
//   6. column / last-axis tables, Green-operator directions, twiddles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <map>
#include <atomic>
#include <cmath>
#include <cstring>
#include <vector>
#include <string>
#include <cstdlib>
#include <thread>

#include "mor_internal.h"

namespace {

struct Dims {
  int32_t nd, n0, n1, n2;
};

// Grids hold at most 2^27 points (checked at plan creation), so 32-bit
// unsigned division suffices (64-bit division is a long instruction sequence).
__device__ __forceinline__ void unravel(const Dims& d, int64_t lin, int* k) {
  const uint32_t l = (uint32_t)lin;
  if (d.nd == 2) {
    k[0] = (int)(l / (uint32_t)d.n1);
    k[1] = (int)(l % (uint32_t)d.n1);
    k[2] = 0;
  } else {
    k[2] = (int)(l % (uint32_t)d.n2);
    const uint32_t r = l / (uint32_t)d.n2;
    k[1] = (int)(r % (uint32_t)d.n1);
    k[0] = (int)(r / (uint32_t)d.n1);
  }
}

__device__ __forceinline__ int64_t ravel(const Dims& d, const int* k) {
  if (d.nd == 2) return (int64_t)k[0] * d.n1 + k[1];
  return ((int64_t)k[0] * d.n1 + k[1]) * d.n2 + k[2];
}

__device__ __forceinline__ int signed_k(int k, int n) { return k <= n / 2 ? k : k - n; }

__device__ __forceinline__ uint32_t lexrank(const Dims& d, const int* k) {
  const int n[3] = {d.n0, d.n1, d.n2};
  uint32_t r = 0;
  for (int a = 0; a < d.nd; ++a) r = r * (uint32_t)n[a] + (uint32_t)(signed_k(k[a], n[a]) + (n[a] - 1) / 2);
  return r;
}

__device__ __forceinline__ void conj_k(const Dims& d, const int* k, int* c) {
  const int n[3] = {d.n0, d.n1, d.n2};
  for (int a = 0; a < 3; ++a) c[a] = a < d.nd ? (n[a] - k[a]) % n[a] : 0;
}

struct SortEl {
  uint32_t a, b, c, idx;
};

__device__ __forceinline__ bool el_less(const SortEl& x, const SortEl& y) {
  if (x.a != y.a) return x.a < y.a;
  if (x.b != y.b) return x.b < y.b;
  return x.c < y.c;
}

// Block-wide exclusive scan of one int per thread (blockDim multiple of 64).
__device__ int block_excl_scan(int v, int* lds, int* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < nw; ++w) {
      int t = lds[w];
      lds[w] = s;
      s += t;
    }
    lds[nw] = s;
  }
  __syncthreads();
  int res = x - v + lds[wid];
  *total = lds[nw];
  __syncthreads();
  return res;
}

// Per-plan device destinations of a batched construction (one entry per
// microstructure; workgroups find theirs from the batch index).
struct PlanPtrs {
  uint8_t* g;
  int64_t* rank;
  int64_t* slot_rep;
  cpx<float>* slot_ghat;
  int64_t* sorted;
  int32_t* ints;
  int64_t* coef_lin;
  float* coef_n;
  double* coef_n64;
  uint8_t* coef_flag;
  int32_t* coef_slot;
  cpx<float>* tw;
  cpx<double>* tw64;
  PlanDev* dev;
  int64_t M, nslots;
  int32_t ncol, nlast;
};

// Offsets of the integer tables inside PlanPtrs::ints (the same for every
// plan of a grid): col_k | col_last | col_off | last_k | last_off | coef_k0.
struct IntLayout {
  int32_t col_k, col_last, col_off, last_k, last_off, coef_k0;
};

template <typename T>
__device__ __forceinline__ cpx<T>* plan_tw(const PlanPtrs& q);
template <>
__device__ __forceinline__ cpx<float>* plan_tw<float>(const PlanPtrs& q) { return q.tw; }
template <>
__device__ __forceinline__ cpx<double>* plan_tw<double>(const PlanPtrs& q) { return q.tw64; }

// ------------------------------------------------------------------ kernels

__global__ void k_twiddle_f64(cpx<double>* tw, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double s, c;
  sincospi(2.0 * (double)t / (double)n, &s, &c);
  tw[t] = {c, -s};
}

// The four solver twiddle tables in one launch, packed tw0 [n0] | tw1 [n1] |
// twh [nh] | rtw [nl], each exp(-2 pi i t / length) evaluated in FP64 (and
// rounded for the FP32 tables).
template <typename T>
__global__ void k_twiddle4(const PlanPtrs* __restrict__ pp, int n0, int n1, int nh, int nl) {
  cpx<T>* __restrict__ tw = plan_tw<T>(pp[blockIdx.y]);
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int n;
  int u = t;
  if (u < n0) {
    n = n0;
  } else if ((u -= n0) < n1) {
    n = n1;
  } else if ((u -= n1) < nh) {
    n = nh;
  } else if ((u -= nh) < nl) {
    n = nl;
  } else {
    return;
  }
  double s, c;
  sincospi(2.0 * (double)u / (double)n, &s, &c);
  tw[t] = {(T)c, (T)(-s)};
}

// Phase maps [batch][N] -> each plan's copy of g and the complex FP64 input
// of the spectrum; blockIdx.y = plan.
__global__ void k_g_to_cplx(const uint8_t* __restrict__ G, const PlanPtrs* __restrict__ pp,
                            cpx<double>* __restrict__ S, int64_t N, unsigned long long* count) {
  const int b = blockIdx.y;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int v = 0;
  if (i < N) {
    v = G[(int64_t)b * N + i];
    pp[b].g[i] = (uint8_t)v;
    S[(int64_t)b * N + i] = {(double)v, 0.0};
  }
  // integer count of inclusion voxels (order-independent, exact): one
  // atomic per workgroup
  __shared__ unsigned int wc[16];
  const unsigned long long m = __ballot(v != 0);
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = (unsigned int)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += wc[w];
    if (t) atomicAdd(count + b, t);
  }
}

// FFT of every line along one axis of a C-ordered complex array viewed as
// [outer][na][inner]; `lpw` lines per workgroup.
__global__ void k_fft_axis_f64(cpx<double>* __restrict__ S, int outer, int na, int inner, int lpw, FftDesc fd,
                               const cpx<double>* __restrict__ tw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  cpx<double>* twl = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* A = twl + na;
  cpx<double>* B = A + lpw * na;
  for (int t = threadIdx.x; t < na; t += blockDim.x) twl[t] = tw[t];
  const int64_t nlines = (int64_t)outer * inner;
  const int64_t l0 = (int64_t)blockIdx.x * lpw;
  for (int t = threadIdx.x; t < lpw * na; t += blockDim.x) {
    int e = t / lpw, q = t - e * lpw;  // q fastest: consecutive lines are adjacent in memory when inner > 1
    int64_t l = l0 + q;
    if (l < nlines) {
      const int64_t o = (int64_t)((uint32_t)l / (uint32_t)inner), i = l - o * inner;  // lines < 2^32
      A[q * na + e] = S[(o * na + e) * inner + i];
    } else {
      A[q * na + e] = {0.0, 0.0};
    }
  }
  __syncthreads();
  cpx<double>* R = fft_stockham<double, -1>(A, B, lpw, na, fd, twl);
  for (int t = threadIdx.x; t < lpw * na; t += blockDim.x) {
    int e = t / lpw, q = t - e * lpw;
    int64_t l = l0 + q;
    if (l < nlines) {
      const int64_t o = (int64_t)((uint32_t)l / (uint32_t)inner), i = l - o * inner;  // lines < 2^32
      S[(o * na + e) * inner + i] = R[q * na + e];
    }
  }
}

// Ranking keys: one SortEl per conjugate pair (its representative), appended
// to `out`, and one per self-conjugate frequency (a member of every axis is 0
// or n/2; 2^ndim of them), appended to `side` (kSide slots per plan).
// blockIdx.y = plan: its spectrum at S + b N, its elements at out + b stride.
constexpr int kSide = 8;

// Fixed radial pattern (Sec. 4.1): L lines through xi = 0 at angles l pi / L
// from the axis-1 direction.  One thread per (line = blockIdx.y, step u along
// the line's major axis); the point on the minor axis is the nearest integer
// (halves away from zero) to u tan(angle).  Marks the frequencies in `mask`
// (one map for the batch: the pattern does not depend on g).  Rounding ties
// do not occur (tan(l pi / L) is irrational unless it is 0 or +-1).
__global__ void k_radial_mark(int n0, int n1, int L, uint8_t* __restrict__ mask) {
  const int l = blockIdx.y;
  const int h0 = n0 / 2 - 1, h1 = n1 / 2 - 1;
  const bool shallow = 4 * l <= L || 4 * l >= 3 * L;  // advances along axis 1
  const int hmaj = shallow ? h1 : h0, hmin = shallow ? h0 : h1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > 2 * hmaj) return;
  const int u = t - hmaj;
  const double ang = shallow ? M_PI * (double)l / (double)L : M_PI * (double)(L - 2 * l) / (2.0 * (double)L);
  const double x = (double)u * tan(ang);
  const double v = copysign(floor(fabs(x) + 0.5), x);
  if (fabs(v) > (double)hmin) return;
  const int iv = (int)v;
  const int s0 = shallow ? iv : u, s1 = shallow ? u : iv;
  mask[(int64_t)((s0 + n0) % n0) * n1 + (s1 + n1) % n1] = 1;
}

// Number of marked frequencies (integer atomics: exact in any order).
__global__ void k_mask_count(const uint8_t* __restrict__ mask, int64_t N, unsigned long long* __restrict__ count) {
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    c += mask[i];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

__global__ __launch_bounds__(256) void k_keys(const cpx<double>* __restrict__ S, Dims d, int64_t N,
                                              const unsigned long long* count, const uint8_t* __restrict__ radial,
                                              SortEl* __restrict__ out, int64_t stride,
                                              const int* __restrict__ blockoff, SortEl* __restrict__ side,
                                              unsigned int* nside) {
  const int b = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = (int)(threadIdx.x & 63);
  S += (int64_t)b * N;
  count += b;
  out += (int64_t)b * stride;
  bool main_rep = false, self_rep = false;
  SortEl e{};
  if (i < N) {
    int k[3], c[3];
    unravel(d, i, k);
    conj_k(d, k, c);
    const uint32_t lr = lexrank(d, k), lc = lexrank(d, c);
    if (lr <= lc) {  // else the partner represents this pair
      const double cnt = (double)(*count);
      const double P0 = cnt * cnt;
      double P;
      if (i == 0) {
        P = P0;
      } else {
        cpx<double> v = S[i];
        P = v.x * v.x + v.y * v.y;
      }
      float key = 0.0f;
      if (radial) {
        key = radial[i] ? 1.0f : 0.0f;  // every frequency of the fixed pattern ranks alike
      } else if (P0 > 0.0 && !(P <= ldexp(P0, -80))) {
        key = (float)(P / P0);
      }
      const int n[3] = {d.n0, d.n1, d.n2};
      uint32_t s2 = 0;
      for (int a = 0; a < d.nd; ++a) {
        int s = signed_k(k[a], n[a]);
        s2 += (uint32_t)(s * s);
      }
      e = {~__float_as_uint(key), s2, lr, (uint32_t)i};
      self_rep = lr == lc;
      main_rep = !self_rep;
    }
  }
  if (self_rep) {  // at most 2^ndim per plan
    const unsigned int pos = atomicAdd(nside + b, 1u);
    side[(int64_t)b * kSide + pos] = e;
  }
  // the pairs' representatives in index order: the block's offset (the
  // same for every plan: which frequencies represent their pair depends on
  // the grid only) plus the place within the block
  __shared__ unsigned int woff[16];
  const unsigned long long m = __ballot(main_rep);
  const int w = (int)(threadIdx.x >> 6);
  if (lane == 0) woff[w] = (unsigned int)__popcll(m);
  __syncthreads();
  unsigned int before = blockoff[blockIdx.x];
  for (int q = 0; q < w; ++q) before += woff[q];
  if (main_rep) out[before + __popcll(m & ((1ull << lane) - 1ull))] = e;
}

// Pair representatives per block of 256 frequencies (the layout of k_keys;
// blockIdx.x = block), for the offsets of k_keys' output.
__global__ __launch_bounds__(256) void k_rep_counts(Dims d, int64_t N, int* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool main_rep = false;
  if (i < N) {
    int k[3], c[3];
    unravel(d, i, k);
    conj_k(d, k, c);
    main_rep = lexrank(d, k) < lexrank(d, c);
  }
  __shared__ unsigned int wc[16];
  const unsigned long long m = __ballot(main_rep);
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = (unsigned int)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int t = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += wc[q];
    cnt[blockIdx.x] = (int)t;
  }
}

// Rank order of every representative of a plan (blockIdx.y): its sorted pairs
// (main, nmain_b[plan] of them) merged with its nside self-conjugate
// frequencies (unsorted, at most kSide).  Keys are a total order, so each element's place
// is its index in its own list plus the count of smaller ones in the other.
__global__ void k_merge_side(const SortEl* __restrict__ main, int64_t stride, const unsigned int* __restrict__ nmain_b,
                             const SortEl* __restrict__ side, int nside, SortEl* __restrict__ out, int64_t nreps) {
  const int b = blockIdx.y;
  const int64_t nmain = nmain_b[b];
  main += (int64_t)b * stride;
  side += (int64_t)b * kSide;
  out += (int64_t)b * nreps;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nmain) {
    const SortEl x = main[i];
    int c = 0;
    for (int t = 0; t < nside; ++t) c += el_less(side[t], x) ? 1 : 0;
    out[i + c] = x;
  } else if (i < nmain + nside) {
    const SortEl x = side[i - nmain];
    int r = 0;
    for (int t = 0; t < nside; ++t) r += el_less(side[t], x) ? 1 : 0;
    int64_t lo = 0, hi = nmain;  // first main element not less than x
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (el_less(main[mid], x)) {
        lo = mid + 1;
      } else {
        hi = mid;
      }
    }
    out[r + lo] = x;
  }
}

// Sentinels (larger than every key) in positions [from_b[plan], to) of each
// plan's segment (blockIdx.y = plan).
__global__ void k_fill_sentinel(SortEl* el, const unsigned int* __restrict__ from_b, int64_t to, int64_t stride) {
  const int64_t i = (int64_t)from_b[blockIdx.y] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < to) el[(int64_t)blockIdx.y * stride + i] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
}

__global__ void k_fill_u32(unsigned int* __restrict__ p, int n, unsigned int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Top-T threshold of every plan's pair representatives (one workgroup per
// plan): the first sort word (inverted key bits) of the T-th smallest
// element, T = ceil(M/2) (no more pairs can be selected), by a radix select
// over 8-bit digits, most significant first.  The elements whose first word
// is at most this value are a superset of the first T in the total order.
__global__ __launch_bounds__(1024) void k_topk_threshold(const SortEl* __restrict__ el, int64_t stride, int64_t nmain,
                                                         const PlanPtrs* __restrict__ pp, uint32_t* __restrict__ thr) {
  __shared__ unsigned int hist[256];
  __shared__ uint32_t s_digit, s_want;
  const int b = blockIdx.x;
  el += (int64_t)b * stride;
  const int64_t T = min((pp[b].M + 1) / 2, nmain);
  uint32_t prefix = 0u, pmask = 0u, want = (uint32_t)max<int64_t>(T, 1);
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int t = threadIdx.x; t < 256; t += blockDim.x) hist[t] = 0u;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < nmain; i += blockDim.x) {
      const uint32_t a = el[i].a;
      if ((a & pmask) == prefix) atomicAdd(&hist[(a >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t cum = 0u, dg = 255u;
      for (uint32_t q = 0; q < 256u; ++q) {
        if (cum + hist[q] >= want) {
          dg = q;
          break;
        }
        cum += hist[q];
      }
      s_digit = dg;
      s_want = want - cum;
    }
    __syncthreads();
    prefix |= s_digit << shift;
    pmask |= 255u << shift;
    want = s_want;
    __syncthreads();
  }
  if (threadIdx.x == 0) thr[b] = prefix;
}

// Candidates of each plan (blockIdx.y): the representatives whose first sort
// word is at most the plan's threshold, gathered into its segment of `cand`
// (one atomic per wavefront claims the slots; the sort that follows fixes
// the order).
__global__ void k_topk_compact(const SortEl* __restrict__ el, int64_t stride, int64_t nmain,
                               const uint32_t* __restrict__ thr, SortEl* __restrict__ cand, int64_t cstride,
                               unsigned int* __restrict__ ccount) {
  const int b = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = (int)(threadIdx.x & 63);
  SortEl e{};
  bool take = false;
  if (i < nmain) {
    e = el[(int64_t)b * stride + i];
    take = e.a <= thr[b];
  }
  const unsigned long long m = __ballot(take);
  if (m) {
    const int first = __ffsll((long long)m) - 1;
    unsigned int base = 0;
    if (lane == first) base = atomicAdd(ccount + b, (unsigned int)__popcll(m));
    base = __shfl(base, first, 64);
    if (take) cand[(int64_t)b * cstride + base + __popcll(m & ((1ull << lane) - 1ull))] = e;
  }
}

// Bitonic network, ascending, over n elements made of independent segments of
// `seg` (a power of two, one per plan): compare-exchange pairs never leave a
// segment (j < k <= seg), and the direction is taken from the index inside
// the segment, so every segment ends sorted ascending.  Global step (k, j).
// Segment s of `seg` elements starts at element s * stride (stride >= seg).
__device__ __forceinline__ int64_t seg_addr(int64_t i, int64_t seg, int64_t stride) {
  return (i / seg) * stride + (i & (seg - 1));
}

__global__ void k_bitonic_global(SortEl* el, int64_t n, int64_t seg, int64_t k, int64_t j, int64_t stride) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // pair index
  if (t >= n / 2) return;
  int64_t i = (t / j) * 2 * j + (t % j);
  int64_t l = i + j;
  bool asc = ((i & (seg - 1)) & k) == 0;
  const int64_t ai = seg_addr(i, seg, stride), al = seg_addr(l, seg, stride);
  SortEl x = el[ai], y = el[al];
  bool sw = asc ? el_less(y, x) : el_less(x, y);
  if (sw) {
    el[ai] = y;
    el[al] = x;
  }
}

// In-LDS part of the network for tiles of `tile` elements (blockDim = tile/2).
// kmin == 0: full local sort of each tile (k = 2 .. tile).  Otherwise: merge
// steps j = tile/2 .. 1 for the given k.
__global__ void k_bitonic_local(SortEl* el, int tile, int64_t seg, int64_t kglob, int64_t stride) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  SortEl* s = reinterpret_cast<SortEl*>(smem_raw);
  const int64_t base = (int64_t)blockIdx.x * tile;
  const int64_t abase = seg_addr(base, seg, stride);  // a tile never straddles segments
  for (int t = threadIdx.x; t < tile; t += blockDim.x) s[t] = el[abase + t];
  __syncthreads();
  auto step = [&](int64_t k, int j) {
    int t = threadIdx.x;
    int i = (t / j) * 2 * j + (t % j);
    int l = i + j;
    bool asc = (((base + i) & (seg - 1)) & k) == 0;
    SortEl x = s[i], y = s[l];
    bool sw = asc ? el_less(y, x) : el_less(x, y);
    if (sw) {
      s[i] = y;
      s[l] = x;
    }
    __syncthreads();
  };
  if (kglob == 0) {
    for (int k = 2; k <= tile; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) step(k, j);
  } else {
    for (int j = tile >> 1; j > 0; j >>= 1) step(kglob, j);
  }
  for (int t = threadIdx.x; t < tile; t += blockDim.x) el[abase + t] = s[t];
}

// Pair-atomic selection in rank order (one workgroup per plan, blockIdx.x).
// Also records, for every selected frequency, its pair index in rank order
// (bit 30 set for the partner of the pair's representative); Mact[1] = number
// of selected pairs.
__global__ void k_select(const SortEl* __restrict__ el, int64_t stride, const unsigned int* __restrict__ nmain_b,
                         int nside, Dims d, int64_t N, const PlanPtrs* __restrict__ pp, uint8_t* __restrict__ mask,
                         int64_t* __restrict__ Mact, int* __restrict__ pairof) {
  __shared__ int lds[32];
  const int b = blockIdx.x;
  const int64_t nreps = (int64_t)nmain_b[b] + nside;
  el += (int64_t)b * stride;
  mask += (int64_t)b * N;
  pairof += (int64_t)b * N;
  Mact += 2 * b;
  const int64_t M = pp[b].M;
  int64_t* __restrict__ rank = pp[b].rank;
  int64_t base = 0;
  for (int64_t c0 = 0; c0 < nreps; c0 += blockDim.x) {
    int64_t i = c0 + threadIdx.x;
    int sz = 0;
    int64_t idx = 0, pidx = 0;
    if (i < nreps) {
      idx = el[i].idx;
      int k[3], c[3];
      unravel(d, idx, k);
      conj_k(d, k, c);
      pidx = ravel(d, c);
      sz = pidx == idx ? 1 : 2;
    }
    int total;
    int ex = block_excl_scan(sz, lds, &total);
    int64_t pos = base + ex;
    if (sz && pos < M) {
      rank[pos] = idx;
      mask[idx] = 1;
      pairof[idx] = (int)i;
      if (sz == 2) {
        rank[pos + 1] = pidx;
        mask[pidx] = 1;
        pairof[pidx] = (int)i | (1 << 30);
      }
      if (pos + sz >= M) {
        Mact[0] = pos + sz;
        Mact[1] = i + 1;
      }
    }
    base += total;
    if (base >= M) break;
  }
}

// Sorted pattern (increasing linear index) in three launches: per-chunk
// counts, an exclusive scan of the counts, and the scatter of each chunk
// (plan = blockIdx.y, for the scan blockIdx.x).
constexpr int kCompactChunk = 4096;

__global__ __launch_bounds__(256) void k_compact_count(const uint8_t* __restrict__ mask, int64_t N,
                                                       int* __restrict__ ccount, int nchunk) {
  __shared__ int lds[32];
  mask += (int64_t)blockIdx.y * N;
  ccount += (int64_t)blockIdx.y * nchunk;
  const int64_t c0 = (int64_t)blockIdx.x * kCompactChunk;
  int n = 0;
  for (int t = threadIdx.x; t < kCompactChunk; t += 256) {
    const int64_t i = c0 + t;
    n += (i < N) ? (int)mask[i] : 0;
  }
  int total;
  (void)block_excl_scan(n, lds, &total);
  if (threadIdx.x == 0) ccount[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_compact_scan(int* __restrict__ ccount, int nchunk) {
  __shared__ int lds[32];
  ccount += (int64_t)blockIdx.x * nchunk;
  int base = 0;
  for (int c0 = 0; c0 < nchunk; c0 += 1024) {
    const int i = c0 + threadIdx.x;
    const int v = i < nchunk ? ccount[i] : 0;
    int total;
    const int ex = block_excl_scan(v, lds, &total);
    if (i < nchunk) ccount[i] = base + ex;
    base += total;
  }
}

__global__ __launch_bounds__(256) void k_compact_scatter(const uint8_t* __restrict__ mask, int64_t N,
                                                         const int* __restrict__ cbase, int nchunk,
                                                         const PlanPtrs* __restrict__ pp) {
  __shared__ int lds[32];
  mask += (int64_t)blockIdx.y * N;
  cbase += (int64_t)blockIdx.y * nchunk;
  int64_t* __restrict__ sorted = pp[blockIdx.y].sorted;
  const int64_t c0 = (int64_t)blockIdx.x * kCompactChunk;
  int base = cbase[blockIdx.x];
  for (int t0 = 0; t0 < kCompactChunk; t0 += 256) {
    const int64_t i = c0 + t0 + threadIdx.x;
    const int f = (i < N) ? (int)mask[i] : 0;
    int total;
    const int ex = block_excl_scan(f, lds, &total);
    if (f) sorted[base + ex] = i;
    base += total;
  }
}

// Slot tables of the warm-start network: slot s = pair s+1 in rank order
// (pair 0 is xi = 0): representative's linear index and g^(rep) / count.
__global__ void k_slots(const SortEl* __restrict__ el, int64_t stride, const cpx<double>* __restrict__ S, int64_t N,
                        const unsigned long long* count, const PlanPtrs* __restrict__ pp) {
  const int b = blockIdx.y;
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= pp[b].nslots) return;
  el += (int64_t)b * stride;
  S += (int64_t)b * N;
  count += b;
  int64_t* __restrict__ slot_rep = pp[b].slot_rep;
  cpx<float>* __restrict__ slot_ghat = pp[b].slot_ghat;
  const int64_t rep = el[s + 1].idx;
  const double c = (double)(*count);
  const cpx<double> v = S[rep];
  slot_rep[s] = rep;
  slot_ghat[s] = c > 0.0 ? cpx<float>{(float)(v.x / c), (float)(v.y / c)} : cpx<float>{0.f, 0.f};
}

// Half-spectrum columns: column c = kh * n1 + k1 (3D) or c = kh (2D), kh the
// last-axis frequency in [0, nlen/2].
__global__ __launch_bounds__(256) void k_tab_count(const uint8_t* __restrict__ mask, Dims d, int64_t N, int ncolall,
                                                   int nkh, int* __restrict__ cnt, int* __restrict__ lastcnt) {
  // one wavefront per column: lanes stride over k0, wavefront sum; plan = blockIdx.y
  const int c = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (c >= ncolall) return;
  mask += (int64_t)blockIdx.y * N;
  cnt += (int64_t)blockIdx.y * ncolall;
  lastcnt += (int64_t)blockIdx.y * nkh;
  int n = 0;
  const int kh = d.nd == 2 ? c : c / d.n1;
  if (d.nd == 2) {
    for (int k0 = lane; k0 < d.n0; k0 += 64) n += mask[(int64_t)k0 * d.n1 + c];
  } else {
    const int k1 = c - kh * d.n1;
    for (int k0 = lane; k0 < d.n0; k0 += 64) n += mask[((int64_t)k0 * d.n1 + k1) * d.n2 + kh];
  }
  for (int o = 32; o > 0; o >>= 1) n += __shfl_down(n, o, 64);
  if (lane == 0) {
    cnt[c] = n;
    if (n) atomicAdd(&lastcnt[kh], n);
  }
}

// One workgroup per plan (blockIdx.x): column and last-axis indices and offsets.
__global__ void k_tab_scan(const int* __restrict__ cnt, const int* __restrict__ lastcnt, Dims d, int ncolall, int nkh,
                           int* __restrict__ colidx, int* __restrict__ col_kh, int* __restrict__ lastidx,
                           int* __restrict__ meta, const PlanPtrs* __restrict__ pp, IntLayout il) {
  __shared__ int lds[32];
  __shared__ int lds2[32];
  const int b = blockIdx.x;
  cnt += (int64_t)b * ncolall;
  colidx += (int64_t)b * ncolall;
  col_kh += (int64_t)b * ncolall;
  lastcnt += (int64_t)b * nkh;
  lastidx += (int64_t)b * nkh;
  meta += 4 * b;
  int32_t* __restrict__ col_k = pp[b].ints + il.col_k;
  int32_t* __restrict__ col_off = pp[b].ints + il.col_off;
  int32_t* __restrict__ last_k = pp[b].ints + il.last_k;
  int jb = 0, ob = 0;
  for (int c0 = 0; c0 < ncolall; c0 += blockDim.x) {
    int c = c0 + threadIdx.x;
    int n = c < ncolall ? cnt[c] : 0;
    int ne = n > 0;
    int tj, to;
    int j = block_excl_scan(ne, lds, &tj);
    int o = block_excl_scan(n, lds2, &to);
    if (c < ncolall) colidx[c] = ne ? jb + j : -1;
    if (ne) {
      col_off[jb + j] = ob + o;
      col_k[jb + j] = d.nd == 2 ? c : c % d.n1;
      col_kh[jb + j] = d.nd == 2 ? c : c / d.n1;
    }
    jb += tj;
    ob += to;
  }
  if (threadIdx.x == 0) {
    col_off[jb] = ob;
    meta[0] = jb;  // ncol
    meta[2] = ob;  // ncoef
  }
  int lb = 0;
  for (int c0 = 0; c0 < nkh; c0 += blockDim.x) {
    int c = c0 + threadIdx.x;
    int ne = c < nkh ? lastcnt[c] > 0 : 0;
    int tl;
    int j = block_excl_scan(ne, lds, &tl);
    if (c < nkh) lastidx[c] = ne ? lb + j : -1;
    if (ne) last_k[lb + j] = c;
    lb += tl;
  }
  if (threadIdx.x == 0) meta[1] = lb;  // nlast
}

__global__ void k_tab_groups(const int* __restrict__ col_kh, const int* __restrict__ lastidx, int ncolall, int nkh,
                             const PlanPtrs* __restrict__ pp, IntLayout il) {
  const int b = blockIdx.y;
  const int ncol = pp[b].ncol, nlast = pp[b].nlast;
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > ncol) return;
  col_kh += (int64_t)b * ncolall;
  lastidx += (int64_t)b * nkh;
  int32_t* __restrict__ col_last = pp[b].ints + il.col_last;
  int32_t* __restrict__ last_off = pp[b].ints + il.last_off;
  if (j == ncol) {
    last_off[nlast] = ncol;
    return;
  }
  int jl = lastidx[col_kh[j]];
  col_last[j] = jl;
  if (j == 0 || lastidx[col_kh[j - 1]] != jl) last_off[jl] = j;
}

// Pattern entries of each column, rows ascending, with Green directions.
__device__ void coef_entry(const uint8_t* __restrict__ mask, Dims d, int gamma_kind, const int* k, int64_t lin, int e,
                           int* __restrict__ coef_k0, int64_t* __restrict__ coef_lin, float* __restrict__ coef_n,
                           double* __restrict__ coef_n64, uint8_t* __restrict__ flag, const int* __restrict__ pairof,
                           int* __restrict__ coef_slot) {
  const int n[3] = {d.n0, d.n1, d.n2};
  coef_k0[e] = k[0];
  coef_lin[e] = lin;
  {
    // slot s = pair - 1 (pair 0 is xi = 0 -> -1); bit 30: stored member is the partner
    const int pr = pairof[lin];
    const int pair = pr & ((1 << 30) - 1);
    coef_slot[e] = pair == 0 ? -1 : ((pair - 1) | (pr & (1 << 30)));
  }
  double v[3] = {0.0, 0.0, 0.0};
  uint8_t f = 0;
  bool zero = true, selfc = true;
  int nyq = 0, nyq_axis = -1;
  for (int a = 0; a < d.nd; ++a) {
    if (k[a] != 0) zero = false;
    bool isn = (n[a] % 2 == 0) && (k[a] == n[a] / 2);
    if (isn) {
      ++nyq;
      nyq_axis = a;
    }
    if (!(k[a] == 0 || isn)) selfc = false;
  }
  if (zero) {
    f = COEF_ZERO;
  } else if (gamma_kind == MOR_GAMMA_ROTATED) {
    if (nyq >= 2) {
      f = COEF_DEAD;
    } else if (nyq == 1) {
      v[nyq_axis] = 1.0;
    } else {
      double nn = 0.0;
      for (int a = 0; a < d.nd; ++a) {
        v[a] = tan(M_PI * (double)k[a] / (double)n[a]);
        nn += v[a] * v[a];
      }
      nn = sqrt(nn);
      for (int a = 0; a < d.nd; ++a) v[a] /= nn;
    }
  } else {
    if (nyq >= 1 && !selfc) {
      f = COEF_DEAD;
    } else {
      double nn = 0.0;
      for (int a = 0; a < d.nd; ++a) {
        v[a] = (double)signed_k(k[a], n[a]);
        nn += v[a] * v[a];
      }
      nn = sqrt(nn);
      for (int a = 0; a < d.nd; ++a) v[a] /= nn;
    }
  }
  coef_n[3 * e + 0] = (float)v[0];
  coef_n[3 * e + 1] = (float)v[1];
  coef_n[3 * e + 2] = (float)v[2];
  coef_n64[3 * e + 0] = v[0];
  coef_n64[3 * e + 1] = v[1];
  coef_n64[3 * e + 2] = v[2];
  flag[e] = f;
}

// Coefficient tables: one wavefront per half-spectrum column c walks k0 in
// chunks of 64; a ballot and the popcount of the lower lanes give each
// selected entry its slot (entries of a column stay in increasing k0).
__global__ __launch_bounds__(256) void k_tab_fill(const uint8_t* __restrict__ mask, Dims d, int64_t N, int ncolall,
                                                  const int* __restrict__ colidx, const int* __restrict__ pairof,
                                                  int gamma_kind, const PlanPtrs* __restrict__ pp, IntLayout il) {
  const int c = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (c >= ncolall) return;
  const int b = blockIdx.y;
  mask += (int64_t)b * N;
  pairof += (int64_t)b * N;
  colidx += (int64_t)b * ncolall;
  const PlanPtrs& q = pp[b];
  const int32_t* __restrict__ col_off = q.ints + il.col_off;
  int32_t* __restrict__ coef_k0 = q.ints + il.coef_k0;
  int64_t* __restrict__ coef_lin = q.coef_lin;
  float* __restrict__ coef_n = q.coef_n;
  double* __restrict__ coef_n64 = q.coef_n64;
  uint8_t* __restrict__ flag = q.coef_flag;
  int32_t* __restrict__ coef_slot = q.coef_slot;
  const int j = colidx[c];
  if (j < 0) return;
  int e = col_off[j];
  int kh, k1;
  if (d.nd == 2) {
    kh = c;
    k1 = c;
  } else {
    kh = c / d.n1;
    k1 = c - kh * d.n1;
  }
  for (int base = 0; base < d.n0; base += 64) {
    const int k0 = base + lane;
    int k[3];
    k[0] = k0;
    if (d.nd == 2) {
      k[1] = kh;
      k[2] = 0;
    } else {
      k[1] = k1;
      k[2] = kh;
    }
    const int64_t lin = k0 < d.n0 ? ravel(d, k) : 0;
    const bool sel = k0 < d.n0 && mask[lin];
    const unsigned long long bal = __ballot(sel);
    if (sel) {
      const int pos = __popcll(bal & ((1ull << lane) - 1ull));
      coef_entry(mask, d, gamma_kind, k, lin, e + pos, coef_k0, coef_lin, coef_n, coef_n64, flag, pairof,
                 coef_slot);
    }
    e += __popcll(bal);
  }
}

// Each plan's PlanDev from an array staged in device memory (blockIdx.x = plan).
static_assert(sizeof(PlanDev) % 4 == 0, "PlanDev is copied in 4-byte words");
__global__ void k_put_plandev(const PlanDev* __restrict__ src, const PlanPtrs* __restrict__ pp) {
  const int b = blockIdx.x;
  const uint32_t* __restrict__ from = reinterpret_cast<const uint32_t*>(src + b);
  uint32_t* __restrict__ to = reinterpret_cast<uint32_t*>(pp[b].dev);
  for (int w = threadIdx.x; w < (int)(sizeof(PlanDev) / 4); w += blockDim.x) to[w] = from[w];
}

bool size_ok(int64_t n) {
  if (n < 4 || n > 1024 || (n % 2)) return false;
  FftDesc d;
  return fft_make_desc((int)n, &d) && fft_make_desc((int)(n / 2), &d);
}

template <typename T>
struct DevBuf {
  T* p = nullptr;
  hipError_t alloc(struct PlanScratch& sc, size_t n);
};

// Temporaries of plan construction come from a per-device pool of device
// blocks that are kept for reuse (plan construction is called once per
// microstructure, often thousands of times; hipMalloc/hipFree pairs dominated
// its cost).  A PlanScratch hands out blocks for one construction and gives
// them back when it ends, after draining the stream.
struct ScratchPool {
  std::mutex mu;
  std::multimap<size_t, void*> free;  // size -> block
};

ScratchPool& scratch_pool(int dev) {
  static std::mutex mu;
  static std::map<int, ScratchPool*> pools;
  std::lock_guard<std::mutex> lk(mu);
  auto it = pools.find(dev);
  if (it != pools.end()) return *it->second;
  ScratchPool* p = new ScratchPool();
  pools[dev] = p;
  return *p;
}

struct PlanScratch {
  hipStream_t st;
  int dev = 0;
  std::vector<std::pair<size_t, void*>> held;
  explicit PlanScratch(hipStream_t s) : st(s) { (void)hipGetDevice(&dev); }
  hipError_t get(void** out, size_t bytes) {
    bytes = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
    ScratchPool& pool = scratch_pool(dev);
    {
      std::lock_guard<std::mutex> lk(pool.mu);
      auto it = pool.free.lower_bound(bytes);
      if (it != pool.free.end() && it->first <= 4 * bytes) {
        held.push_back(*it);
        *out = it->second;
        pool.free.erase(it);
        return hipSuccess;
      }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return e;
    held.push_back({bytes, p});
    *out = p;
    return hipSuccess;
  }
  ~PlanScratch() {
    (void)hipStreamSynchronize(st);  // queued kernels may still use the blocks
    ScratchPool& pool = scratch_pool(dev);
    std::lock_guard<std::mutex> lk(pool.mu);
    for (auto& h : held) pool.free.insert(h);
  }
};

template <typename T>
hipError_t DevBuf<T>::alloc(PlanScratch& sc, size_t n) {
  return sc.get((void**)&p, std::max<size_t>(n, 1) * sizeof(T));
}

}  // namespace

static void plan_free(mor_plan* p) {
  if (!p) return;
  if (!p->blocks.empty()) {
    // the blocks go back to the pool: nothing queued may still use them
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != p->device) (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    if (cur != p->device) (void)hipSetDevice(cur);
    ScratchPool& pool = scratch_pool(p->device);
    std::lock_guard<std::mutex> lk(pool.mu);
    for (auto& b : p->blocks) pool.free.insert(b);
  }
  delete p;
}

// Pinned host staging of a batch's phase maps.  Buffers are kept in a
// per-device free list for reuse (allocating and freeing pinned memory can
// stall the whole device, which a plan construction overlapped with solves
// on another stream must not do); one is handed back after its stream has
// drained (the copy from it is asynchronous).
struct PinnedPool {
  std::mutex mu;
  std::multimap<size_t, void*> free;
};
PinnedPool& pinned_pool(int dev) {
  static std::mutex mu;
  static std::map<int, PinnedPool*> pools;
  std::lock_guard<std::mutex> lk(mu);
  auto it = pools.find(dev);
  if (it != pools.end()) return *it->second;
  PinnedPool* p = new PinnedPool();
  pools[dev] = p;
  return *p;
}

struct PinnedStage {
  hipStream_t st;
  int dev = 0;
  void* p = nullptr;
  size_t bytes = 0;
  explicit PinnedStage(hipStream_t s) : st(s) { (void)hipGetDevice(&dev); }
  hipError_t get(size_t want) {
    PinnedPool& pool = pinned_pool(dev);
    {
      std::lock_guard<std::mutex> lk(pool.mu);
      auto it = pool.free.lower_bound(want);
      if (it != pool.free.end()) {
        bytes = it->first;
        p = it->second;
        pool.free.erase(it);
        return hipSuccess;
      }
    }
    bytes = want;
    return hipHostMalloc(&p, want, hipHostMallocDefault);
  }
  ~PinnedStage() {
    if (p) {
      (void)hipStreamSynchronize(st);
      PinnedPool& pool = pinned_pool(dev);
      std::lock_guard<std::mutex> lk(pool.mu);
      pool.free.insert({bytes, p});
    }
  }
};

// Device blocks of a batch of plans: each from the pool when one fits, the
// others carved from one allocation (one hipMalloc per batch, not per plan);
// the carved pieces go back to the pool like any block and are never freed.
static hipError_t plan_alloc_batch(mor_plan* const* P, int cnt, const std::vector<size_t>& sizes,
                                   std::vector<unsigned char*>& bases) {
  bases.assign(cnt, nullptr);
  std::vector<int> miss;
  size_t total = 0;
  ScratchPool& pool = scratch_pool(P[0]->device);
  {
    std::lock_guard<std::mutex> lk(pool.mu);
    for (int b = 0; b < cnt; ++b) {
      const size_t bytes = (std::max<size_t>(sizes[b], 1) + 255) / 256 * 256;
      auto it = pool.free.lower_bound(bytes);
      if (it != pool.free.end() && it->first <= 4 * bytes) {
        P[b]->blocks.push_back(*it);
        bases[b] = (unsigned char*)it->second;
        pool.free.erase(it);
      } else {
        miss.push_back(b);
        total += bytes;
      }
    }
  }
  if (miss.empty()) return hipSuccess;
  unsigned char* slab = nullptr;
  const hipError_t e = hipMalloc((void**)&slab, total);
  if (e != hipSuccess) return e;
  size_t at = 0;
  for (int b : miss) {
    const size_t bytes = (std::max<size_t>(sizes[b], 1) + 255) / 256 * 256;
    bases[b] = slab + at;
    P[b]->blocks.push_back({bytes, slab + at});
    at += bytes;
  }
  return hipSuccess;
}

// Host work over `n` items split across threads when it is large (map
// checks and staging copies of big batches); fn(begin, end) handles a range.
template <typename F>
static void host_parallel(int64_t n, size_t bytes, F fn) {
  const unsigned hc = std::max(1u, std::thread::hardware_concurrency());
  const int64_t nt = std::min<int64_t>({(int64_t)std::min(hc, 8u), n, (int64_t)(bytes >> 22) + 1});
  if (nt <= 1) {
    fn((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  const int64_t per = (n + nt - 1) / nt;
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t a = t * per, b = std::min(n, a + per);
    if (a < b) th.emplace_back(fn, a, b);
  }
  for (auto& x : th) x.join();
}

// Builds `cnt` plans of one grid (P[i]->M may differ) from host phase maps
// maps[0..cnt) (each N bytes, already checked), staged through `pinned`
// (cnt N bytes of pinned host memory, or NULL to copy the maps one by one).
// Every step is one launch over the whole batch (plan = a grid dimension of
// the launch), with two host synchronisations for the sizes of the per-plan
// tables.  Scratch: about 30 N + 16 N' bytes per plan (N' the power of two at
// or above the number of conjugate pairs).
static mor_status plan_build_batch(mor_plan* const* P, const int cnt, const uint8_t* const* maps, uint8_t* pinned,
                                   hipStream_t st) {
  PlanScratch sc(st);  // declared first: released last, after the stream has drained
  const mor_plan& P0 = *P[0];
  const int nd = P0.ndim;
  const int64_t N = P0.N;
  Dims d{nd, P0.n[0], P0.n[1], nd == 3 ? P0.n[2] : 1};
  const int nlen = nd == 2 ? P0.n[1] : P0.n[2];
  const unsigned nb = (unsigned)cnt;

  // Radial pattern: the lines do not depend on g, so one map serves the
  // batch; its size fixes M (whole conjugate pairs by construction).
  DevBuf<uint8_t> radial;
  if (P0.pattern_kind == MOR_PATTERN_RADIAL) {
    DevBuf<unsigned long long> rc;
    MOR_HIP_TRY(radial.alloc(sc, (size_t)N));
    MOR_HIP_TRY(rc.alloc(sc, 1));
    MOR_HIP_TRY(hipMemsetAsync(radial.p, 0, (size_t)N, st));
    MOR_HIP_TRY(hipMemsetAsync(rc.p, 0, sizeof(unsigned long long), st));
    const int hmax = std::max(P0.n[0], P0.n[1]) / 2 - 1;
    k_radial_mark<<<dim3((unsigned)((2 * hmax + 1 + 255) / 256), (unsigned)P0.radial_lines), 256, 0, st>>>(
        P0.n[0], P0.n[1], P0.radial_lines, radial.p);
    MOR_LAUNCH_CHECK("radial_mark");
    k_mask_count<<<(unsigned)std::min<int64_t>(1024, (N + 255) / 256), 256, 0, st>>>(radial.p, N, rc.p);
    MOR_LAUNCH_CHECK("mask_count");
    unsigned long long hc = 0;
    MOR_HIP_TRY(hipMemcpyAsync(&hc, rc.p, sizeof(hc), hipMemcpyDeviceToHost, st));
    MOR_HIP_TRY(hipStreamSynchronize(st));
    if (hc < 1 || (int64_t)hc > N) {
      mor_set_error("mor_plan: radial pattern size outside [1, N]");
      return MOR_E_DEVICE;
    }
    for (int b = 0; b < cnt; ++b) P[b]->M = (int64_t)hc;
  }

  std::vector<PlanPtrs> hp(cnt);
  DevBuf<PlanPtrs> pp;
  DevBuf<uint8_t> G;
  MOR_HIP_TRY(pp.alloc(sc, cnt));
  MOR_HIP_TRY(G.alloc(sc, (size_t)cnt * N));
  // The maps reach the device in one copy from the pinned staging buffer (a
  // host memcpy of each, then one DMA; the previous chunk's copy has drained
  // at its final synchronisation), else one copy per map.
  if (pinned) {
    host_parallel(cnt, (size_t)cnt * N, [&](int64_t a, int64_t e) {
      for (int64_t b = a; b < e; ++b) std::memcpy(pinned + (size_t)b * N, maps[b], (size_t)N);
    });
    MOR_HIP_TRY(hipMemcpyAsync(G.p, pinned, (size_t)cnt * N, hipMemcpyHostToDevice, st));
  } else {
    for (int b = 0; b < cnt; ++b)
      MOR_HIP_TRY(hipMemcpyAsync(G.p + (size_t)b * N, maps[b], N, hipMemcpyHostToDevice, st));
  }
  // Every device table of a plan lives in one block of the pool, laid out
  // with upper bounds known before the selection: M_actual <= M + 1, and the
  // selected pairs, slots and stored coefficients are at most M_actual.
  const int nkh = nlen / 2 + 1;
  const int ncolall = nd == 2 ? nkh : nkh * P0.n[1];
  const int64_t cap_col = ncolall, cap_last = nkh;
  IntLayout il;
  il.col_k = 0;
  il.col_last = (int32_t)cap_col;
  il.col_off = (int32_t)(2 * cap_col);
  il.last_k = (int32_t)(3 * cap_col + 1);
  il.last_off = (int32_t)(3 * cap_col + 1 + cap_last);
  il.coef_k0 = (int32_t)(3 * cap_col + 1 + 2 * cap_last + 1);
  const int n0 = P0.n[0], n1 = P0.n[1];
  const int ntw = n0 + n1 + nlen / 2 + nlen;
  // layout of every plan's block (offsets within it), then the blocks
  struct Layout {
    size_t g, rank, srep, sghat, sorted, ints, clin, cn, cn64, flag, slot, tw, tw64, dev, total;
  };
  std::vector<Layout> lay(cnt);
  std::vector<size_t> sizes(cnt);
  for (int b = 0; b < cnt; ++b) {
    const int64_t m1 = P[b]->M + 1;
    size_t at = 0;
    auto take = [&at](size_t bytes) {
      const size_t o = at;
      at += (bytes + 255) / 256 * 256;
      return o;
    };
    Layout& L = lay[b];
    L.g = take(N);
    L.rank = take(m1 * 8);
    L.srep = take(m1 * 8);
    L.sghat = take(m1 * 8);
    L.sorted = take(m1 * 8);
    L.ints = take((il.coef_k0 + m1) * 4);
    L.clin = take(m1 * 8);
    L.cn = take(m1 * 12);
    L.cn64 = take(m1 * 24);
    L.flag = take(m1);
    L.slot = take(m1 * 4);
    L.tw = take(ntw * sizeof(cpx<float>));
    L.tw64 = take(ntw * sizeof(cpx<double>));
    L.dev = take(sizeof(PlanDev));
    L.total = at;
    sizes[b] = at;
  }
  std::vector<unsigned char*> bases;
  MOR_HIP_TRY(plan_alloc_batch(P, cnt, sizes, bases));
  for (int b = 0; b < cnt; ++b) {
    mor_plan* Q = P[b];
    const Layout& L = lay[b];
    const size_t o_g = L.g, o_rank = L.rank, o_srep = L.srep, o_sghat = L.sghat, o_sorted = L.sorted,
                 o_ints = L.ints, o_clin = L.clin, o_cn = L.cn, o_cn64 = L.cn64, o_flag = L.flag, o_slot = L.slot,
                 o_tw = L.tw, o_tw64 = L.tw64, o_dev = L.dev;
    unsigned char* base = bases[b];
    Q->d_g = base + o_g;
    Q->d_rank = (int64_t*)(base + o_rank);
    Q->d_slot_rep = (int64_t*)(base + o_srep);
    Q->d_slot_ghat = (cpx<float>*)(base + o_sghat);
    Q->d_sorted = (int64_t*)(base + o_sorted);
    Q->d_ints = (int32_t*)(base + o_ints);
    Q->d_coef_lin = (int64_t*)(base + o_clin);
    Q->d_coef_n = (float*)(base + o_cn);
    Q->d_coef_n64 = (double*)(base + o_cn64);
    Q->d_coef_flag = base + o_flag;
    Q->d_coef_slot = (int32_t*)(base + o_slot);
    Q->d_tw = (cpx<float>*)(base + o_tw);
    Q->d_tw64 = (cpx<double>*)(base + o_tw64);
    Q->d_dev = (PlanDev*)(base + o_dev);
    PlanPtrs& h = hp[b];
    h = PlanPtrs{};
    h.g = Q->d_g;
    h.rank = Q->d_rank;
    h.slot_rep = Q->d_slot_rep;
    h.slot_ghat = Q->d_slot_ghat;
    h.sorted = Q->d_sorted;
    h.ints = Q->d_ints;
    h.coef_lin = Q->d_coef_lin;
    h.coef_n = Q->d_coef_n;
    h.coef_n64 = Q->d_coef_n64;
    h.coef_flag = Q->d_coef_flag;
    h.coef_slot = Q->d_coef_slot;
    h.tw = Q->d_tw;
    h.tw64 = Q->d_tw64;
    h.dev = Q->d_dev;
    h.M = Q->M;
  }
  MOR_HIP_TRY(hipMemcpyAsync(pp.p, hp.data(), cnt * sizeof(PlanPtrs), hipMemcpyHostToDevice, st));

  // 1. FP64 spectrum of every phase map ([cnt][N], each axis batched as lines)
  DevBuf<cpx<double>> S;
  DevBuf<cpx<double>> tw64;
  DevBuf<unsigned long long> count;
  MOR_HIP_TRY(S.alloc(sc, (size_t)cnt * N));
  MOR_HIP_TRY(tw64.alloc(sc, 1024));
  MOR_HIP_TRY(count.alloc(sc, cnt));
  MOR_HIP_TRY(hipMemsetAsync(count.p, 0, cnt * sizeof(unsigned long long), st));
  k_g_to_cplx<<<dim3((unsigned)((N + 255) / 256), nb), 256, 0, st>>>(G.p, pp.p, S.p, N, count.p);
  MOR_LAUNCH_CHECK("g_to_cplx");
  for (int a = 0; a < nd; ++a) {
    int na = P0.n[a];
    int outer = cnt, inner = 1;
    for (int b = 0; b < a; ++b) outer *= P0.n[b];
    for (int b = a + 1; b < nd; ++b) inner *= P0.n[b];
    FftDesc fd;
    fft_make_desc(na, &fd);
    k_twiddle_f64<<<(na + 255) / 256, 256, 0, st>>>(tw64.p, na);
    MOR_LAUNCH_CHECK("twiddle_f64");
    int lpw = std::max(1, 1024 / na);
    int64_t nlines = (int64_t)outer * inner;
    size_t sh = (size_t)(na + 2 * lpw * na) * sizeof(cpx<double>);
    k_fft_axis_f64<<<(unsigned)((nlines + lpw - 1) / lpw), 256, sh, st>>>(S.p, outer, na, inner, lpw, fd, tw64.p);
    MOR_LAUNCH_CHECK("fft_axis_f64");
  }

  // 2. keys: the conjugate pairs' representatives in one segment of npow2
  // elements per plan (sorted below), the self-conjugate frequencies aside
  // (for grids of 2^k points the pairs then fill N/2 slots, not N)
  int64_t nselfc = 1;
  for (int a = 0; a < nd; ++a) nselfc *= 2;  // every axis is even
  const int64_t nmain = (N - nselfc) / 2;
  int64_t npow2 = 1;
  while (npow2 < nmain) npow2 <<= 1;
  const int64_t nel = (int64_t)cnt * npow2;
  DevBuf<SortEl> el, side, ranked, cand;
  DevBuf<unsigned int> nout, ccount;
  DevBuf<uint32_t> thr;
  MOR_HIP_TRY(el.alloc(sc, nel));
  MOR_HIP_TRY(side.alloc(sc, (size_t)cnt * kSide));
  MOR_HIP_TRY(nout.alloc(sc, 2 * (size_t)cnt));
  MOR_HIP_TRY(ccount.alloc(sc, (size_t)cnt));
  MOR_HIP_TRY(thr.alloc(sc, (size_t)cnt));
  MOR_HIP_TRY(hipMemsetAsync(nout.p, 0, 2 * cnt * sizeof(unsigned int), st));
  {
    const int nkb = (int)((N + 255) / 256);
    DevBuf<int> boff;
    MOR_HIP_TRY(boff.alloc(sc, (size_t)nkb));
    k_rep_counts<<<nkb, 256, 0, st>>>(d, N, boff.p);
    MOR_LAUNCH_CHECK("rep_counts");
    k_compact_scan<<<1, 1024, 0, st>>>(boff.p, nkb);  // exclusive scan: block offsets
    MOR_LAUNCH_CHECK("rep_scan");
    k_keys<<<dim3((unsigned)nkb, nb), 256, 0, st>>>(S.p, d, N, count.p, radial.p, el.p, npow2, boff.p, side.p,
                                                    nout.p + cnt);
    MOR_LAUNCH_CHECK("keys");
  }

  // 3. order of the pairs.  No more than T = ceil(M/2) pairs can be
  // selected, so only the candidates for the first T places are sorted: a
  // radix select finds the T-th smallest first sort word, the elements at or
  // below it are gathered and sorted.  When the candidates are not much
  // fewer than all pairs (large M, or many equal keys at the cut) every pair
  // is sorted instead.  Either way the rank order of the selected pairs is
  // the total order of all pairs.
  k_topk_threshold<<<nb, 1024, 0, st>>>(el.p, npow2, nmain, pp.p, thr.p);
  MOR_LAUNCH_CHECK("topk_threshold");
  MOR_HIP_TRY(cand.alloc(sc, nel));
  MOR_HIP_TRY(hipMemsetAsync(ccount.p, 0, cnt * sizeof(unsigned int), st));
  k_topk_compact<<<dim3((unsigned)((nmain + 255) / 256), nb), 256, 0, st>>>(el.p, npow2, nmain, thr.p, cand.p, npow2,
                                                                             ccount.p);
  MOR_LAUNCH_CHECK("topk_compact");
  std::vector<unsigned int> hcc((size_t)cnt);
  MOR_HIP_TRY(hipMemcpyAsync(hcc.data(), ccount.p, cnt * sizeof(unsigned int), hipMemcpyDeviceToHost, st));
  MOR_HIP_TRY(hipStreamSynchronize(st));
  int64_t maxc = 0;
  for (int b = 0; b < cnt; ++b) maxc = std::max<int64_t>(maxc, hcc[b]);
  int64_t cpow2 = 1;
  while (cpow2 < maxc) cpow2 <<= 1;
  SortEl* keys = cand.p;  // the sorted segments, stride npow2
  int64_t seg = cpow2;
  unsigned int* nsorted = ccount.p;
  if (2 * cpow2 > npow2) {  // not worth it: sort every pair
    keys = el.p;
    seg = npow2;
    k_fill_u32<<<(cnt + 255) / 256, 256, 0, st>>>(ccount.p, cnt, (unsigned int)nmain);
    MOR_LAUNCH_CHECK("fill_counts");
  }
  k_fill_sentinel<<<dim3((unsigned)((seg + 255) / 256), nb), 256, 0, st>>>(keys, nsorted, seg, npow2);
  MOR_LAUNCH_CHECK("fill_sentinel");
  const int64_t nsort = (int64_t)cnt * seg;
  const int tile = (int)std::min<int64_t>(seg, 2048);
  const unsigned nt = (unsigned)std::max(1, tile / 2);
  if (seg >= 2) {
    const unsigned ntiles = (unsigned)(nsort / tile);
    const unsigned npairb = (unsigned)((nsort / 2 + 255) / 256);
    k_bitonic_local<<<ntiles, nt, tile * sizeof(SortEl), st>>>(keys, tile, seg, 0, npow2);
    MOR_LAUNCH_CHECK("bitonic_local");
    for (int64_t k = 2 * (int64_t)tile; k <= seg; k <<= 1) {
      for (int64_t j = k >> 1; j >= tile; j >>= 1) {
        k_bitonic_global<<<npairb, 256, 0, st>>>(keys, nsort, seg, k, j, npow2);
        MOR_LAUNCH_CHECK("bitonic_global");
      }
      k_bitonic_local<<<ntiles, nt, tile * sizeof(SortEl), st>>>(keys, tile, seg, k, npow2);
      MOR_LAUNCH_CHECK("bitonic_local");
    }
  }
  const int64_t nrank = seg + nselfc;  // per-plan stride of the rank order
  MOR_HIP_TRY(ranked.alloc(sc, (size_t)cnt * nrank));
  k_merge_side<<<dim3((unsigned)((nrank + 255) / 256), nb), 256, 0, st>>>(keys, npow2, nsorted, side.p, (int)nselfc,
                                                                          ranked.p, nrank);
  MOR_LAUNCH_CHECK("merge_side");

  // 4. selection
  DevBuf<uint8_t> mask;
  DevBuf<int64_t> mact;
  DevBuf<int> pairof;
  MOR_HIP_TRY(mask.alloc(sc, (size_t)cnt * N));
  MOR_HIP_TRY(mact.alloc(sc, 2 * (size_t)cnt));
  MOR_HIP_TRY(pairof.alloc(sc, (size_t)cnt * N));
  MOR_HIP_TRY(hipMemsetAsync(mask.p, 0, (size_t)cnt * N, st));
  MOR_HIP_TRY(hipMemsetAsync(pairof.p, 0, (size_t)cnt * N * sizeof(int), st));
  k_select<<<nb, 1024, 0, st>>>(ranked.p, nrank, nsorted, (int)nselfc, d, N, pp.p, mask.p, mact.p, pairof.p);
  MOR_LAUNCH_CHECK("select");
  std::vector<int64_t> hm(2 * (size_t)cnt);
  std::vector<unsigned long long> hcount(cnt);
  MOR_HIP_TRY(hipMemcpyAsync(hm.data(), mact.p, 2 * cnt * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MOR_HIP_TRY(hipMemcpyAsync(hcount.data(), count.p, cnt * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  MOR_HIP_TRY(hipStreamSynchronize(st));

  // sizes of the selection
  int64_t max_slots = 0;
  for (int b = 0; b < cnt; ++b) {
    mor_plan* Q = P[b];
    Q->M_actual = hm[2 * b];
    Q->nslots = hm[2 * b + 1] - 1;
    Q->count = (int64_t)hcount[b];
    if (Q->M_actual < 1 || Q->M_actual > Q->M + 1 || Q->nslots < 0 || Q->nslots >= Q->M_actual) {
      mor_set_error("mor_plan: selection sizes outside their bounds");
      return MOR_E_DEVICE;
    }
    max_slots = std::max(max_slots, Q->nslots);
    hp[b].nslots = Q->nslots;
  }
  MOR_HIP_TRY(hipMemcpyAsync(pp.p, hp.data(), cnt * sizeof(PlanPtrs), hipMemcpyHostToDevice, st));

  // slot tables of the warm-start network
  if (max_slots > 0) {
    k_slots<<<dim3((unsigned)((max_slots + 255) / 256), nb), 256, 0, st>>>(ranked.p, nrank, S.p, N, count.p, pp.p);
    MOR_LAUNCH_CHECK("slots");
  }

  // 5. sorted pattern
  {
    const int nchunk = (int)((N + kCompactChunk - 1) / kCompactChunk);
    DevBuf<int> ccount;
    MOR_HIP_TRY(ccount.alloc(sc, (size_t)cnt * nchunk));
    k_compact_count<<<dim3(nchunk, nb), 256, 0, st>>>(mask.p, N, ccount.p, nchunk);
    k_compact_scan<<<nb, 1024, 0, st>>>(ccount.p, nchunk);
    k_compact_scatter<<<dim3(nchunk, nb), 256, 0, st>>>(mask.p, N, ccount.p, nchunk, pp.p);
    MOR_LAUNCH_CHECK("compact");
  }

  // 6. tables
  DevBuf<int> cntc, lastcnt, colidx, col_kh, lastidx, meta;
  MOR_HIP_TRY(cntc.alloc(sc, (size_t)cnt * ncolall));
  MOR_HIP_TRY(lastcnt.alloc(sc, (size_t)cnt * nkh));
  MOR_HIP_TRY(colidx.alloc(sc, (size_t)cnt * ncolall));
  MOR_HIP_TRY(col_kh.alloc(sc, (size_t)cnt * ncolall));
  MOR_HIP_TRY(lastidx.alloc(sc, (size_t)cnt * nkh));
  MOR_HIP_TRY(meta.alloc(sc, 4 * (size_t)cnt));
  MOR_HIP_TRY(hipMemsetAsync(lastcnt.p, 0, (size_t)cnt * nkh * sizeof(int), st));
  k_tab_count<<<dim3((ncolall + 3) / 4, nb), 256, 0, st>>>(mask.p, d, N, ncolall, nkh, cntc.p, lastcnt.p);
  MOR_LAUNCH_CHECK("tab_count");
  k_tab_scan<<<nb, 1024, 0, st>>>(cntc.p, lastcnt.p, d, ncolall, nkh, colidx.p, col_kh.p, lastidx.p, meta.p, pp.p, il);
  MOR_LAUNCH_CHECK("tab_scan");
  std::vector<int> hmeta(4 * (size_t)cnt);
  MOR_HIP_TRY(hipMemcpyAsync(hmeta.data(), meta.p, 4 * cnt * sizeof(int), hipMemcpyDeviceToHost, st));
  MOR_HIP_TRY(hipStreamSynchronize(st));

  int max_col = 0;
  std::vector<PlanDev> hdev(cnt);
  for (int b = 0; b < cnt; ++b) {
    mor_plan* Q = P[b];
    const int ncol = hmeta[4 * b], nlast = hmeta[4 * b + 1], ncoef = hmeta[4 * b + 2];
    max_col = std::max(max_col, ncol);
    if (ncol < 0 || ncol > ncolall || nlast < 0 || nlast > nkh || ncoef < 0 || ncoef > Q->M_actual) {
      mor_set_error("mor_plan: table sizes outside their bounds");
      return MOR_E_DEVICE;
    }
    hp[b].ncol = ncol;
    hp[b].nlast = nlast;

    PlanDev& v = Q->dev;
    v = PlanDev{};
    v.ndim = nd;
    v.n0 = n0;
    v.n1 = n1;
    v.n2 = nd == 3 ? P0.n[2] : 1;
    v.N = (int32_t)N;
    v.nlen = nlen;
    v.rows = (int32_t)(N / nlen);
    v.ncol = ncol;
    v.nlast = nlast;
    v.ncoef = ncoef;
    v.inv_N = (float)(1.0 / (double)N);
    v.g = Q->d_g;
    v.col_k = Q->d_ints + il.col_k;
    v.col_last = Q->d_ints + il.col_last;
    v.col_off = Q->d_ints + il.col_off;
    v.last_k = Q->d_ints + il.last_k;
    v.last_off = Q->d_ints + il.last_off;
    v.coef_k0 = Q->d_ints + il.coef_k0;
    v.coef_n = Q->d_coef_n;
    v.coef_flag = Q->d_coef_flag;
    v.tw0 = Q->d_tw;
    v.tw1 = v.tw0 + n0;
    v.twh = v.tw1 + n1;
    v.rtw = v.twh + nlen / 2;
    v.coef_n64 = Q->d_coef_n64;
    v.tw0_64 = Q->d_tw64;
    v.tw1_64 = v.tw0_64 + n0;
    v.twh_64 = v.tw1_64 + n1;
    v.rtw_64 = v.twh_64 + nlen / 2;
    fft_make_desc(n0, &v.fd0);
    fft_make_desc(n1, &v.fd1);
    fft_make_desc(nlen / 2, &v.fdh);
    hdev[b] = v;
  }
  MOR_HIP_TRY(hipMemcpyAsync(pp.p, hp.data(), cnt * sizeof(PlanPtrs), hipMemcpyHostToDevice, st));
  k_tab_groups<<<dim3((max_col + 1 + 255) / 256, nb), 256, 0, st>>>(col_kh.p, lastidx.p, ncolall, nkh, pp.p, il);
  MOR_LAUNCH_CHECK("tab_groups");
  k_tab_fill<<<dim3((ncolall + 3) / 4, nb), 256, 0, st>>>(mask.p, d, N, ncolall, colidx.p, pairof.p, P0.gamma_kind,
                                                          pp.p, il);
  MOR_LAUNCH_CHECK("tab_fill");

  // twiddles of the solver transforms, and each plan's device descriptor
  k_twiddle4<float><<<dim3((ntw + 255) / 256, nb), 256, 0, st>>>(pp.p, n0, n1, nlen / 2, nlen);
  MOR_LAUNCH_CHECK("twiddle_f32");
  k_twiddle4<double><<<dim3((ntw + 255) / 256, nb), 256, 0, st>>>(pp.p, n0, n1, nlen / 2, nlen);
  MOR_LAUNCH_CHECK("twiddle_f64");
  DevBuf<PlanDev> dstage;
  MOR_HIP_TRY(dstage.alloc(sc, cnt));
  MOR_HIP_TRY(hipMemcpyAsync(dstage.p, hdev.data(), cnt * sizeof(PlanDev), hipMemcpyHostToDevice, st));
  k_put_plandev<<<nb, 64, 0, st>>>(dstage.p, pp.p);
  MOR_LAUNCH_CHECK("put_plandev");
  MOR_HIP_TRY(hipStreamSynchronize(st));
  return MOR_OK;
}

// Scratch bytes of one plan in plan_build_batch.
static size_t plan_scratch_bytes(const mor_grid* grid, int64_t N) {
  int64_t nselfc = 1;
  for (int a = 0; a < grid->ndim; ++a) nselfc *= 2;
  const int64_t nmain = (N - nselfc) / 2;
  int64_t npow2 = 1;
  while (npow2 < nmain) npow2 <<= 1;
  const int64_t nlen = grid->n[grid->ndim - 1];
  const int64_t ncolall = (nlen / 2 + 1) * (grid->ndim == 3 ? grid->n[1] : 1);
  // keys and candidates (16 npow2 each), the rank order (at most npow2 +
  // 2^ndim entries), spectrum, masks and tables
  return (size_t)(22 * N + 48 * npow2 + 16 * nselfc + 16 * kSide + 12 * ncolall + 8 * (nlen / 2 + 1) +
                  4 * (N / 4096 + 1) + 16 + sizeof(PlanPtrs) + sizeof(PlanDev) + 64);
}

// Shared by mor_plan_create (count 1) and mor_plan_create_batch.
static mor_status plan_create_n(const char* who, const mor_grid* grid, int64_t count, const uint8_t* const* maps,
                                const int64_t* Ms, const mor_plan_opts* opts, mor_plan_t* out) {
  if (!grid || (count > 0 && (!maps || !Ms || !out))) {
    mor_set_error(std::string(who) + ": NULL argument");
    return MOR_E_INVALID_ARG;
  }
  if (count < 0) {
    mor_set_error(std::string(who) + ": negative count");
    return MOR_E_INVALID_ARG;
  }
  for (int64_t b = 0; b < count; ++b) out[b] = nullptr;
  if (grid->ndim != 2 && grid->ndim != 3) {
    mor_set_error(std::string(who) + ": ndim must be 2 or 3");
    return MOR_E_INVALID_ARG;
  }
  int64_t N = 1;
  for (int a = 0; a < grid->ndim; ++a) {
    if (grid->n[a] < 2) {
      mor_set_error(std::string(who) + ": every grid size must be >= 2");
      return MOR_E_INVALID_ARG;
    }
    N *= grid->n[a];
  }
  for (int a = 0; a < grid->ndim; ++a) {
    if (!size_ok(grid->n[a])) {
      mor_set_error(std::string(who) + ": grid sizes must be even, 2^a 3^b, within [4, 1024]");
      return MOR_E_UNSUPPORTED;
    }
  }
  if (N > (int64_t)1 << 27) {
    mor_set_error(std::string(who) + ": grid larger than 2^27 points");
    return MOR_E_UNSUPPORTED;
  }
  for (int64_t b = 0; b < count; ++b) {
    if (Ms[b] < 1 || Ms[b] > N) {
      mor_set_error(std::string(who) + ": M must lie in [1, N] (microstructure " + std::to_string(b) + ")");
      return MOR_E_INVALID_ARG;
    }
  }
  int gk = opts ? opts->gamma_kind : MOR_GAMMA_ROTATED;
  if (gk != MOR_GAMMA_ROTATED && gk != MOR_GAMMA_CONTINUOUS) {
    mor_set_error(std::string(who) + ": unknown gamma_kind");
    return MOR_E_INVALID_ARG;
  }
  const int pk = opts ? opts->pattern_kind : MOR_PATTERN_ADAPTED;
  const int lines = opts ? opts->radial_lines : 0;
  if (pk != MOR_PATTERN_ADAPTED && pk != MOR_PATTERN_RADIAL) {
    mor_set_error(std::string(who) + ": unknown pattern_kind");
    return MOR_E_INVALID_ARG;
  }
  if (pk == MOR_PATTERN_RADIAL) {
    if (grid->ndim != 2) {
      mor_set_error(std::string(who) + ": the radial pattern is defined for 2D grids");
      return MOR_E_UNSUPPORTED;
    }
    if (lines < 1 || lines > 4096) {
      mor_set_error(std::string(who) + ": radial_lines must lie in [1, 4096]");
      return MOR_E_INVALID_ARG;
    }
  }
  for (int64_t b = 0; b < count; ++b) {
    if (!maps[b]) {
      mor_set_error(std::string(who) + ": NULL phase map (microstructure " + std::to_string(b) + ")");
      return MOR_E_INVALID_ARG;
    }
  }
  // every value 0 or 1: the OR of a map's bytes is above 1 iff some value is
  std::vector<uint8_t> bad((size_t)count, 0);
  host_parallel(count, (size_t)count * N, [&](int64_t a, int64_t e) {
    for (int64_t b = a; b < e; ++b) {
      const uint8_t* g = maps[b];
      uint8_t any = 0;
      for (int64_t i = 0; i < N; ++i) any |= g[i];
      bad[b] = any > 1;
    }
  });
  for (int64_t b = 0; b < count; ++b) {
    if (bad[b]) {
      mor_set_error(std::string(who) + ": phase_map values must be 0 or 1 (microstructure " + std::to_string(b) + ")");
      return MOR_E_INVALID_ARG;
    }
  }
  if (count == 0) return MOR_OK;

  size_t budget = (size_t)512 << 20;
  if (const char* e = getenv("MOR_PLAN_SCRATCH_BYTES")) {
    long long v = atoll(e);
    if (v > 0) budget = (size_t)v;
  }
  const int64_t chunk =
      std::max<int64_t>(1, std::min<int64_t>({count, (int64_t)(budget / plan_scratch_bytes(grid, N)), 65535}));

  static std::atomic<uint64_t> next_uid{0};
  std::vector<mor_plan*> P((size_t)count, nullptr);
  int dev = 0;
  (void)hipGetDevice(&dev);
  for (int64_t b = 0; b < count; ++b) {
    mor_plan* Q = new mor_plan();
    Q->uid = ++next_uid;
    Q->ndim = grid->ndim;
    for (int a = 0; a < grid->ndim; ++a) Q->n[a] = (int)grid->n[a];
    Q->N = N;
    Q->M = Ms[b];
    Q->gamma_kind = gk;
    Q->pattern_kind = pk;
    Q->radial_lines = pk == MOR_PATTERN_RADIAL ? lines : 0;
    Q->device = dev;
    P[b] = Q;
  }
  hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
  mor_status s = MOR_OK;
  PinnedStage stage(st);
  if (count > 1) {
    const hipError_t e = stage.get((size_t)chunk * N);
    if (e != hipSuccess) {
      stage.p = nullptr;
      mor_set_error(std::string(who) + ": pinned staging buffer: " + hipGetErrorString(e));
      s = e == hipErrorOutOfMemory ? MOR_E_OUT_OF_MEMORY : MOR_E_DEVICE;
    }
  }
  for (int64_t b0 = 0; b0 < count && s == MOR_OK; b0 += chunk) {
    const int n = (int)std::min<int64_t>(chunk, count - b0);
    s = plan_build_batch(P.data() + b0, n, maps + b0, (uint8_t*)stage.p, st);
  }
  if (s != MOR_OK) {
    (void)hipStreamSynchronize(st);
    for (mor_plan* Q : P) plan_free(Q);
    return s;
  }
  for (int64_t b = 0; b < count; ++b) out[b] = P[b];
  return MOR_OK;
}

extern "C" mor_status mor_plan_create(const mor_grid* grid, const uint8_t* phase_map, int64_t M,
                                      const mor_plan_opts* opts, mor_plan_t* out) {
  if (!grid || !phase_map || !out) {
    mor_set_error("mor_plan_create: NULL argument");
    return MOR_E_INVALID_ARG;
  }
  const uint8_t* const maps[1] = {phase_map};
  return plan_create_n("mor_plan_create", grid, 1, maps, &M, opts, out);
}

extern "C" mor_status mor_plan_create_batch(const mor_grid* grid, int64_t count, const uint8_t* const* phase_maps,
                                            const int64_t* M, const mor_plan_opts* opts, mor_plan_t* out) {
  return plan_create_n("mor_plan_create_batch", grid, count, phase_maps, M, opts, out);
}

extern "C" mor_status mor_plan_get_info(mor_plan_t plan, mor_plan_info* info) {
  if (!plan || !info) {
    mor_set_error("mor_plan_get_info: NULL argument");
    return MOR_E_INVALID_ARG;
  }
  info->N = plan->N;
  info->M = plan->M;
  info->M_actual = plan->M_actual;
  info->n_coeff = plan->dev.ncoef;
  info->n_columns = plan->dev.ncol;
  info->n_last = plan->dev.nlast;
  info->inclusion_count = plan->count;
  info->ncomp = plan->ndim == 2 ? 3 : 6;
  info->nstress = plan->ndim == 2 ? 4 : 6;
  info->pattern_kind = plan->pattern_kind;
  info->radial_lines = plan->radial_lines;
  return MOR_OK;
}

extern "C" mor_status mor_plan_pattern(mor_plan_t plan, int64_t* sorted_idx, int64_t* rank_idx, int64_t cap,
                                       int64_t* M_actual) {
  if (!plan) {
    mor_set_error("mor_plan_pattern: NULL plan");
    return MOR_E_INVALID_ARG;
  }
  if (M_actual) *M_actual = plan->M_actual;
  if ((sorted_idx || rank_idx) && cap < plan->M_actual) {
    mor_set_error("mor_plan_pattern: cap < M_actual");
    return MOR_E_INVALID_ARG;
  }
  if (sorted_idx)
    MOR_HIP_TRY(hipMemcpy(sorted_idx, plan->d_sorted, plan->M_actual * sizeof(int64_t), hipMemcpyDeviceToHost));
  if (rank_idx)
    MOR_HIP_TRY(hipMemcpy(rank_idx, plan->d_rank, plan->M_actual * sizeof(int64_t), hipMemcpyDeviceToHost));
  return MOR_OK;
}

extern "C" mor_status mor_plan_coeff_index(mor_plan_t plan, int64_t* lin_idx, int64_t cap) {
  if (!plan || !lin_idx) {
    mor_set_error("mor_plan_coeff_index: NULL argument");
    return MOR_E_INVALID_ARG;
  }
  if (cap < plan->dev.ncoef) {
    mor_set_error("mor_plan_coeff_index: cap < n_coeff");
    return MOR_E_INVALID_ARG;
  }
  MOR_HIP_TRY(hipMemcpy(lin_idx, plan->d_coef_lin, plan->dev.ncoef * sizeof(int64_t), hipMemcpyDeviceToHost));
  return MOR_OK;
}

extern "C" mor_status mor_plan_destroy(mor_plan_t plan) {
  if (!plan) return MOR_OK;
  (void)hipDeviceSynchronize();
  plan_free(plan);
  return MOR_OK;
}
