// Adapted sampling pattern and plan tables (paper Sec. 4.2; reduced scheme of
// Sec. 4).  Every step runs on the device:
//   1. FP64 FFT of the phase indicator g (Stockham along each axis),
//   2. per-frequency ranking keys and pair representatives,
//   3. bitonic sort of the representatives by (key desc, |s|^2, lexrank),
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

#include "mor_internal.h"

namespace {

struct Dims {
  int32_t nd, n0, n1, n2;
};

__device__ __forceinline__ void unravel(const Dims& d, int64_t lin, int* k) {
  if (d.nd == 2) {
    k[0] = (int)(lin / d.n1);
    k[1] = (int)(lin % d.n1);
    k[2] = 0;
  } else {
    k[2] = (int)(lin % d.n2);
    int64_t r = lin / d.n2;
    k[1] = (int)(r % d.n1);
    k[0] = (int)(r / d.n1);
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
__global__ void k_twiddle4(cpx<T>* tw, int n0, int n1, int nh, int nl) {
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

__global__ void k_g_to_cplx(const uint8_t* __restrict__ g, cpx<double>* __restrict__ S, int64_t N,
                            unsigned long long* count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int v = 0;
  if (i < N) {
    v = g[i];
    S[i] = {(double)v, 0.0};
  }
  // integer count of inclusion voxels (order-independent, exact)
  unsigned long long b = __ballot(v != 0);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (unsigned long long)__popcll(b));
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
      int64_t o = l / inner, i = l - o * inner;
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
      int64_t o = l / inner, i = l - o * inner;
      S[(o * na + e) * inner + i] = R[q * na + e];
    }
  }
}

// Ranking keys; appends one SortEl per conjugate pair (its representative).
__global__ void k_keys(const cpx<double>* __restrict__ S, Dims d, int64_t N, const unsigned long long* count,
                       SortEl* __restrict__ out, unsigned int* nout) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int k[3], c[3];
  unravel(d, i, k);
  conj_k(d, k, c);
  uint32_t lr = lexrank(d, k), lc = lexrank(d, c);
  if (lr > lc) return;  // the partner represents this pair
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
  if (P0 > 0.0 && !(P <= ldexp(P0, -80))) key = (float)(P / P0);
  const int n[3] = {d.n0, d.n1, d.n2};
  uint32_t s2 = 0;
  for (int a = 0; a < d.nd; ++a) {
    int s = signed_k(k[a], n[a]);
    s2 += (uint32_t)(s * s);
  }
  unsigned int pos = atomicAdd(nout, 1u);
  out[pos] = {~__float_as_uint(key), s2, lr, (uint32_t)i};
}

__global__ void k_fill_sentinel(SortEl* el, int64_t from, int64_t to) {
  int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < to) el[i] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
}

// Bitonic network, ascending.  Global compare-exchange step (k, j).
__global__ void k_bitonic_global(SortEl* el, int64_t n, int64_t k, int64_t j) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // pair index
  if (t >= n / 2) return;
  int64_t i = (t / j) * 2 * j + (t % j);
  int64_t l = i + j;
  bool asc = (i & k) == 0;
  SortEl x = el[i], y = el[l];
  bool sw = asc ? el_less(y, x) : el_less(x, y);
  if (sw) {
    el[i] = y;
    el[l] = x;
  }
}

// In-LDS part of the network for tiles of `tile` elements (blockDim = tile/2).
// kmin == 0: full local sort of each tile (k = 2 .. tile).  Otherwise: merge
// steps j = tile/2 .. 1 for the given k.
__global__ void k_bitonic_local(SortEl* el, int tile, int64_t kglob) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  SortEl* s = reinterpret_cast<SortEl*>(smem_raw);
  const int64_t base = (int64_t)blockIdx.x * tile;
  for (int t = threadIdx.x; t < tile; t += blockDim.x) s[t] = el[base + t];
  __syncthreads();
  auto step = [&](int64_t k, int j) {
    int t = threadIdx.x;
    int i = (t / j) * 2 * j + (t % j);
    int l = i + j;
    bool asc = ((base + i) & k) == 0;
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
  for (int t = threadIdx.x; t < tile; t += blockDim.x) el[base + t] = s[t];
}

// Pair-atomic selection in rank order (single workgroup).  Also records, for
// every selected frequency, its pair index in rank order (bit 30 set for the
// partner of the pair's representative); Mact[1] = number of selected pairs.
__global__ void k_select(const SortEl* __restrict__ el, int64_t nreps, Dims d, int64_t M, uint8_t* __restrict__ mask,
                         int64_t* __restrict__ rank, int64_t* __restrict__ Mact, int* __restrict__ pairof) {
  __shared__ int lds[32];
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

// Mask -> ascending linear indices (single workgroup).
// Sorted pattern (increasing linear index) in three launches: per-chunk
// counts, an exclusive scan of the counts, and the scatter of each chunk.
constexpr int kCompactChunk = 4096;

__global__ __launch_bounds__(256) void k_compact_count(const uint8_t* __restrict__ mask, int64_t N,
                                                       int* __restrict__ ccount) {
  __shared__ int lds[32];
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
                                                         const int* __restrict__ cbase, int64_t* __restrict__ sorted) {
  __shared__ int lds[32];
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
__global__ void k_slots(const SortEl* __restrict__ el, int64_t nslots, const cpx<double>* __restrict__ S,
                        const unsigned long long* count, int64_t* __restrict__ slot_rep, cpx<float>* __restrict__ slot_ghat) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  const int64_t rep = el[s + 1].idx;
  const double c = (double)(*count);
  const cpx<double> v = S[rep];
  slot_rep[s] = rep;
  slot_ghat[s] = c > 0.0 ? cpx<float>{(float)(v.x / c), (float)(v.y / c)} : cpx<float>{0.f, 0.f};
}

// Half-spectrum columns: column c = kh * n1 + k1 (3D) or c = kh (2D), kh the
// last-axis frequency in [0, nlen/2].
__global__ __launch_bounds__(256) void k_tab_count(const uint8_t* __restrict__ mask, Dims d, int ncolall,
                                                   int* __restrict__ cnt, int* __restrict__ lastcnt) {
  // one wavefront per column: lanes stride over k0, wavefront sum
  const int c = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (c >= ncolall) return;
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

// Single workgroup: column and last-axis indices and offsets.
__global__ void k_tab_scan(const int* __restrict__ cnt, const int* __restrict__ lastcnt, Dims d, int ncolall, int nkh,
                           int* __restrict__ colidx, int* __restrict__ col_k, int* __restrict__ col_kh,
                           int* __restrict__ col_off, int* __restrict__ lastidx, int* __restrict__ last_k,
                           int* __restrict__ meta) {
  __shared__ int lds[32];
  __shared__ int lds2[32];
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

__global__ void k_tab_groups(const int* __restrict__ col_kh, const int* __restrict__ lastidx, int ncol, int nlast,
                             int* __restrict__ col_last, int* __restrict__ last_off) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > ncol) return;
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
__global__ __launch_bounds__(256) void k_tab_fill(const uint8_t* __restrict__ mask, Dims d, int ncolall,
                                                  const int* __restrict__ colidx, const int* __restrict__ col_off,
                                                  int gamma_kind, int* __restrict__ coef_k0,
                                                  int64_t* __restrict__ coef_lin, float* __restrict__ coef_n,
                                                  double* __restrict__ coef_n64, uint8_t* __restrict__ flag,
                                                  const int* __restrict__ pairof, int* __restrict__ coef_slot) {
  const int c = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (c >= ncolall) return;
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

// A device block owned by the plan, from the same pool; plan_free gives the
// plan's blocks back once the device has drained.
template <typename T>
hipError_t plan_alloc(mor_plan* P, T** out, size_t bytes) {
  bytes = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
  ScratchPool& pool = scratch_pool(P->device);
  {
    std::lock_guard<std::mutex> lk(pool.mu);
    auto it = pool.free.lower_bound(bytes);
    if (it != pool.free.end() && it->first <= 4 * bytes) {
      P->blocks.push_back(*it);
      *out = (T*)it->second;
      pool.free.erase(it);
      return hipSuccess;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return e;
  P->blocks.push_back({bytes, p});
  *out = (T*)p;
  return hipSuccess;
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

static mor_status plan_build(mor_plan* P, const uint8_t* phase_map, hipStream_t st) {
  PlanScratch sc(st);  // declared first: released last, after the stream has drained
  const int nd = P->ndim;
  const int64_t N = P->N;
  Dims d{nd, P->n[0], P->n[1], nd == 3 ? P->n[2] : 1};
  const int nlen = nd == 2 ? P->n[1] : P->n[2];

  MOR_HIP_TRY(plan_alloc(P, &P->d_g, N));
  MOR_HIP_TRY(hipMemcpyAsync(P->d_g, phase_map, N, hipMemcpyHostToDevice, st));

  // 1. FP64 spectrum
  DevBuf<cpx<double>> S;
  DevBuf<cpx<double>> tw64;
  DevBuf<unsigned long long> cnt;
  MOR_HIP_TRY(S.alloc(sc, N));
  MOR_HIP_TRY(tw64.alloc(sc, 1024));
  MOR_HIP_TRY(cnt.alloc(sc, 1));
  MOR_HIP_TRY(hipMemsetAsync(cnt.p, 0, sizeof(unsigned long long), st));
  k_g_to_cplx<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(P->d_g, S.p, N, cnt.p);
  MOR_LAUNCH_CHECK("g_to_cplx");
  for (int a = 0; a < nd; ++a) {
    int na = P->n[a];
    int outer = 1, inner = 1;
    for (int b = 0; b < a; ++b) outer *= P->n[b];
    for (int b = a + 1; b < nd; ++b) inner *= P->n[b];
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

  // 2. keys of pair representatives
  int64_t nselfc = 1;
  for (int a = 0; a < nd; ++a) nselfc *= 2;  // every axis is even
  const int64_t nreps = (N + nselfc) / 2;
  int64_t npow2 = 1;
  while (npow2 < nreps) npow2 <<= 1;
  DevBuf<SortEl> el;
  DevBuf<unsigned int> nout;
  MOR_HIP_TRY(el.alloc(sc, npow2));
  MOR_HIP_TRY(nout.alloc(sc, 1));
  MOR_HIP_TRY(hipMemsetAsync(nout.p, 0, sizeof(unsigned int), st));
  k_keys<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(S.p, d, N, cnt.p, el.p, nout.p);
  MOR_LAUNCH_CHECK("keys");
  if (npow2 > nreps) {
    k_fill_sentinel<<<(unsigned)((npow2 - nreps + 255) / 256), 256, 0, st>>>(el.p, nreps, npow2);
    MOR_LAUNCH_CHECK("fill_sentinel");
  }

  // 3. bitonic sort
  const int tile = (int)std::min<int64_t>(npow2, 2048);
  const unsigned nt = (unsigned)std::max(1, tile / 2);
  if (npow2 >= 2) {
    k_bitonic_local<<<(unsigned)(npow2 / tile), nt, tile * sizeof(SortEl), st>>>(el.p, tile, 0);
    MOR_LAUNCH_CHECK("bitonic_local");
    for (int64_t k = 2 * (int64_t)tile; k <= npow2; k <<= 1) {
      for (int64_t j = k >> 1; j >= tile; j >>= 1) {
        k_bitonic_global<<<(unsigned)((npow2 / 2 + 255) / 256), 256, 0, st>>>(el.p, npow2, k, j);
        MOR_LAUNCH_CHECK("bitonic_global");
      }
      k_bitonic_local<<<(unsigned)(npow2 / tile), nt, tile * sizeof(SortEl), st>>>(el.p, tile, k);
      MOR_LAUNCH_CHECK("bitonic_local");
    }
  }

  // 4. selection
  DevBuf<uint8_t> mask;
  DevBuf<int64_t> mact;
  MOR_HIP_TRY(mask.alloc(sc, N));
  MOR_HIP_TRY(mact.alloc(sc, 2));
  MOR_HIP_TRY(hipMemsetAsync(mask.p, 0, N, st));
  MOR_HIP_TRY(plan_alloc(P, &P->d_rank, (P->M + 1) * sizeof(int64_t)));
  DevBuf<int> pairof;
  MOR_HIP_TRY(pairof.alloc(sc, N));
  MOR_HIP_TRY(hipMemsetAsync(pairof.p, 0, N * sizeof(int), st));
  k_select<<<1, 1024, 0, st>>>(el.p, nreps, d, P->M, mask.p, P->d_rank, mact.p, pairof.p);
  MOR_LAUNCH_CHECK("select");
  int64_t hm[2] = {0, 0};
  MOR_HIP_TRY(hipMemcpyAsync(hm, mact.p, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MOR_HIP_TRY(hipMemcpyAsync(&P->count, cnt.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MOR_HIP_TRY(hipStreamSynchronize(st));
  P->M_actual = hm[0];
  P->nslots = hm[1] - 1;

  // slot tables of the warm-start network
  MOR_HIP_TRY(plan_alloc(P, &P->d_slot_rep, std::max<int64_t>(P->nslots, 1) * sizeof(int64_t)));
  MOR_HIP_TRY(plan_alloc(P, &P->d_slot_ghat, std::max<int64_t>(P->nslots, 1) * sizeof(cpx<float>)));
  if (P->nslots > 0) {
    k_slots<<<(unsigned)((P->nslots + 255) / 256), 256, 0, st>>>(el.p, P->nslots, S.p, cnt.p, P->d_slot_rep,
                                                                 P->d_slot_ghat);
    MOR_LAUNCH_CHECK("slots");
  }

  // 5. sorted pattern
  MOR_HIP_TRY(plan_alloc(P, &P->d_sorted, P->M_actual * sizeof(int64_t)));
  {
    const int nchunk = (int)((N + kCompactChunk - 1) / kCompactChunk);
    DevBuf<int> ccount;
    MOR_HIP_TRY(ccount.alloc(sc, nchunk));
    k_compact_count<<<nchunk, 256, 0, st>>>(mask.p, N, ccount.p);
    k_compact_scan<<<1, 1024, 0, st>>>(ccount.p, nchunk);
    k_compact_scatter<<<nchunk, 256, 0, st>>>(mask.p, N, ccount.p, P->d_sorted);
    MOR_LAUNCH_CHECK("compact");
  }

  // 6. tables
  const int nkh = nlen / 2 + 1;
  const int ncolall = nd == 2 ? nkh : nkh * P->n[1];
  DevBuf<int> cntc, lastcnt, colidx, col_kh, lastidx, meta;
  MOR_HIP_TRY(cntc.alloc(sc, ncolall));
  MOR_HIP_TRY(lastcnt.alloc(sc, nkh));
  MOR_HIP_TRY(colidx.alloc(sc, ncolall));
  MOR_HIP_TRY(col_kh.alloc(sc, ncolall));
  MOR_HIP_TRY(lastidx.alloc(sc, nkh));
  MOR_HIP_TRY(meta.alloc(sc, 4));
  MOR_HIP_TRY(hipMemsetAsync(lastcnt.p, 0, nkh * sizeof(int), st));
  // integer layout: col_k | col_last | col_off | last_k | last_off | coef_k0
  const int64_t cap_col = ncolall, cap_last = nkh, cap_coef = P->M_actual;
  const int64_t nint = cap_col + cap_col + (cap_col + 1) + cap_last + (cap_last + 1) + cap_coef;
  MOR_HIP_TRY(plan_alloc(P, &P->d_ints, nint * sizeof(int32_t)));
  int32_t* col_k = P->d_ints;
  int32_t* col_last = col_k + cap_col;
  int32_t* col_off = col_last + cap_col;
  int32_t* last_k = col_off + cap_col + 1;
  int32_t* last_off = last_k + cap_last;
  int32_t* coef_k0 = last_off + cap_last + 1;
  k_tab_count<<<(ncolall + 3) / 4, 256, 0, st>>>(mask.p, d, ncolall, cntc.p, lastcnt.p);
  MOR_LAUNCH_CHECK("tab_count");
  k_tab_scan<<<1, 1024, 0, st>>>(cntc.p, lastcnt.p, d, ncolall, nkh, colidx.p, col_k, col_kh.p, col_off, lastidx.p,
                                 last_k, meta.p);
  MOR_LAUNCH_CHECK("tab_scan");
  int hmeta[4] = {0, 0, 0, 0};
  MOR_HIP_TRY(hipMemcpyAsync(hmeta, meta.p, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
  MOR_HIP_TRY(hipStreamSynchronize(st));
  const int ncol = hmeta[0], nlast = hmeta[1], ncoef = hmeta[2];
  k_tab_groups<<<(ncol + 1 + 255) / 256, 256, 0, st>>>(col_kh.p, lastidx.p, ncol, nlast, col_last, last_off);
  MOR_LAUNCH_CHECK("tab_groups");
  MOR_HIP_TRY(plan_alloc(P, &P->d_coef_lin, std::max(ncoef, 1) * sizeof(int64_t)));
  MOR_HIP_TRY(plan_alloc(P, &P->d_coef_n, std::max(ncoef, 1) * 3 * sizeof(float)));
  MOR_HIP_TRY(plan_alloc(P, &P->d_coef_n64, std::max(ncoef, 1) * 3 * sizeof(double)));
  MOR_HIP_TRY(plan_alloc(P, &P->d_coef_flag, std::max(ncoef, 1)));
  MOR_HIP_TRY(plan_alloc(P, &P->d_coef_slot, std::max(ncoef, 1) * sizeof(int)));
  k_tab_fill<<<(ncolall + 3) / 4, 256, 0, st>>>(mask.p, d, ncolall, colidx.p, col_off, P->gamma_kind, coef_k0,
                                                    P->d_coef_lin, P->d_coef_n, P->d_coef_n64, P->d_coef_flag,
                                                    pairof.p, P->d_coef_slot);
  MOR_LAUNCH_CHECK("tab_fill");

  // twiddles for the solver transforms
  const int n0 = P->n[0], n1 = P->n[1];
  const int ntw = n0 + n1 + nlen / 2 + nlen;
  MOR_HIP_TRY(plan_alloc(P, &P->d_tw, ntw * sizeof(cpx<float>)));
  cpx<float>* tw0 = P->d_tw;
  cpx<float>* tw1 = tw0 + n0;
  cpx<float>* twh = tw1 + n1;
  cpx<float>* rtw = twh + nlen / 2;
  k_twiddle4<float><<<(ntw + 255) / 256, 256, 0, st>>>(P->d_tw, n0, n1, nlen / 2, nlen);
  MOR_LAUNCH_CHECK("twiddle_f32");
  MOR_HIP_TRY(plan_alloc(P, &P->d_tw64, ntw * sizeof(cpx<double>)));
  k_twiddle4<double><<<(ntw + 255) / 256, 256, 0, st>>>(P->d_tw64, n0, n1, nlen / 2, nlen);
  MOR_LAUNCH_CHECK("twiddle_f64");
  (void)tw0;
  (void)tw1;
  (void)twh;
  (void)rtw;

  PlanDev& v = P->dev;
  v.ndim = nd;
  v.n0 = n0;
  v.n1 = n1;
  v.n2 = nd == 3 ? P->n[2] : 1;
  v.N = (int32_t)N;
  v.nlen = nlen;
  v.rows = (int32_t)(N / nlen);
  v.ncol = ncol;
  v.nlast = nlast;
  v.ncoef = ncoef;
  v.inv_N = (float)(1.0 / (double)N);
  v.g = P->d_g;
  v.col_k = col_k;
  v.col_last = col_last;
  v.col_off = col_off;
  v.last_k = last_k;
  v.last_off = last_off;
  v.coef_k0 = coef_k0;
  v.coef_n = P->d_coef_n;
  v.coef_flag = P->d_coef_flag;
  v.tw0 = tw0;
  v.tw1 = tw1;
  v.twh = twh;
  v.rtw = rtw;
  v.coef_n64 = P->d_coef_n64;
  v.tw0_64 = P->d_tw64;
  v.tw1_64 = v.tw0_64 + n0;
  v.twh_64 = v.tw1_64 + n1;
  v.rtw_64 = v.twh_64 + nlen / 2;
  fft_make_desc(n0, &v.fd0);
  fft_make_desc(n1, &v.fd1);
  fft_make_desc(nlen / 2, &v.fdh);
  MOR_HIP_TRY(plan_alloc(P, &P->d_dev, sizeof(PlanDev)));
  MOR_HIP_TRY(hipMemcpyAsync(P->d_dev, &v, sizeof(PlanDev), hipMemcpyHostToDevice, st));
  MOR_HIP_TRY(hipStreamSynchronize(st));
  return MOR_OK;
}

extern "C" mor_status mor_plan_create(const mor_grid* grid, const uint8_t* phase_map, int64_t M,
                                      const mor_plan_opts* opts, mor_plan_t* out) {
  if (!grid || !phase_map || !out) {
    mor_set_error("mor_plan_create: NULL argument");
    return MOR_E_INVALID_ARG;
  }
  *out = nullptr;
  if (grid->ndim != 2 && grid->ndim != 3) {
    mor_set_error("mor_plan_create: ndim must be 2 or 3");
    return MOR_E_INVALID_ARG;
  }
  int64_t N = 1;
  for (int a = 0; a < grid->ndim; ++a) {
    if (grid->n[a] < 2) {
      mor_set_error("mor_plan_create: every grid size must be >= 2");
      return MOR_E_INVALID_ARG;
    }
    N *= grid->n[a];
  }
  for (int a = 0; a < grid->ndim; ++a) {
    if (!size_ok(grid->n[a])) {
      mor_set_error("mor_plan_create: grid sizes must be even, 2^a 3^b, within [4, 1024]");
      return MOR_E_UNSUPPORTED;
    }
  }
  if (N > (int64_t)1 << 27) {
    mor_set_error("mor_plan_create: grid larger than 2^27 points");
    return MOR_E_UNSUPPORTED;
  }
  if (M < 1 || M > N) {
    mor_set_error("mor_plan_create: M must lie in [1, N]");
    return MOR_E_INVALID_ARG;
  }
  int gk = opts ? opts->gamma_kind : MOR_GAMMA_ROTATED;
  if (gk != MOR_GAMMA_ROTATED && gk != MOR_GAMMA_CONTINUOUS) {
    mor_set_error("mor_plan_create: unknown gamma_kind");
    return MOR_E_INVALID_ARG;
  }
  for (int64_t i = 0; i < N; ++i) {
    if (phase_map[i] > 1) {
      mor_set_error("mor_plan_create: phase_map values must be 0 or 1");
      return MOR_E_INVALID_ARG;
    }
  }
  static std::atomic<uint64_t> next_uid{0};
  mor_plan* P = new mor_plan();
  P->uid = ++next_uid;
  P->ndim = grid->ndim;
  for (int a = 0; a < grid->ndim; ++a) P->n[a] = (int)grid->n[a];
  P->N = N;
  P->M = M;
  P->gamma_kind = gk;
  (void)hipGetDevice(&P->device);
  hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
  mor_status s = plan_build(P, phase_map, st);
  if (s != MOR_OK) {
    (void)hipStreamSynchronize(st);
    plan_free(P);
    return s;
  }
  *out = P;
  return MOR_OK;
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
