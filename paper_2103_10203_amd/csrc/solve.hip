// Host driver of the reduced fixed-point iteration: argument checks,
// per-stream workspaces, grouping of RVEs by grid, the iteration loop with
// device-side convergence (the host only polls a counter every few
// iterations), finalisation, load paths and per-kernel profiling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "dft_kernels.h"
#include "solve_fast.h"

using namespace mor_k;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;
void mor_set_error(const std::string& msg) { g_last_error = msg; }
extern "C" const char* mor_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* mor_version(void) { return "mor 0.1 (gfx950)"; }

// ------------------------------------------------------------------ profiling
namespace {
struct ProfStat {
  double ms = 0.0;
  int64_t launches = 0;
  int64_t items = 0;
  double bytes = 0.0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
ProfStat g_prof[PK_COUNT];
const char* kPkName[PK_COUNT] = {"row", "col", "mid_fwd", "mid_inv", "final", "init"};

struct EventPair {
  hipEvent_t a, b;
  int kind;
};

// ------------------------------------------------------------------ workspace
struct Workspace {
  std::map<std::string, std::pair<void*, size_t>> bufs;
  unsigned int* h_active = nullptr;  // pinned
  hipStream_t cap = nullptr;         // private stream for hipGraph capture
  std::vector<hipEvent_t> evpool;
  size_t evnext = 0;
  // Pinned host staging of the solve's small transfers (plan table, offsets,
  // states, effective stresses): copies from pinned memory are queued without
  // a host-side staging copy.  Sized to the largest total one solve asked for,
  // up to kPinStageMax (the first solve of a new size, and whatever does not
  // fit, stages through pageable memory instead); pin_ev follows the last copy
  // that used it.
  unsigned char* pin = nullptr;
  size_t pin_cap = 0, pin_need = 0;
  hipEvent_t pin_ev = nullptr;
  bool pin_busy = false;
  ~Workspace() {}
  template <typename T>
  mor_status get(const char* name, size_t count, T** out) {
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    auto it = bufs.find(name);
    if (it != bufs.end() && it->second.second >= bytes) {
      *out = reinterpret_cast<T*>(it->second.first);
      return MOR_OK;
    }
    if (it != bufs.end()) {
      (void)hipFree(it->second.first);
      bufs.erase(it);
    }
    void* p = nullptr;
    size_t alloc = bytes + bytes / 4;
    if (hipMalloc(&p, alloc) != hipSuccess) {
      (void)hipGetLastError();
      mor_set_error(std::string("workspace allocation failed: ") + name);
      return MOR_E_OUT_OF_MEMORY;
    }
    bufs[name] = {p, alloc};
    *out = reinterpret_cast<T*>(p);
    return MOR_OK;
  }
  hipStream_t capture_stream() {
    if (!cap) (void)hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    return cap;
  }
  hipEvent_t event() {
    if (evnext == evpool.size()) {
      hipEvent_t e;
      (void)hipEventCreate(&e);
      evpool.push_back(e);
    }
    return evpool[evnext++];
  }
};

std::mutex g_ws_mu;
std::map<std::pair<int, void*>, Workspace*> g_ws;

Workspace* workspace_for(void* stream) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto key = std::make_pair(dev, stream);
  auto it = g_ws.find(key);
  if (it != g_ws.end()) return it->second;
  Workspace* w = new Workspace();
  (void)hipHostMalloc((void**)&w->h_active, 64, hipHostMallocDefault);
  g_ws[key] = w;
  return w;
}

// Launch geometry from an LDS budget (bytes).
constexpr int kLdsBudget = 56 * 1024;
// Blocks of the generic kernels within the LDS budget; es = bytes per complex.
int rows_per_block(int C, int nlen, int es = 8) {
  const int nh = nlen / 2;
  int rb = (kLdsBudget / es - (2 * nh + 1)) / (2 * C * (nh + 1));
  return std::max(1, rb);
}
int cols_per_block(int C, int n0, int es = 8) {
  int cb = (kLdsBudget / es - n0) / (2 * C * n0);
  return std::max(1, cb);
}

struct Group {
  int ndim, n0, n1, n2;
  std::vector<int> rves;
  int ncol_max = 0, nlast_max = 0;
  int rb = 1, cb = 1, xb = 1;
  int rvar = 0;  // row-kernel variant
  int cvar = 0;  // column-kernel variant
  int gidx = 0;  // position of the group (active count slot)
  int* d_alist = nullptr;  // this group's segment of the active list
  bool fast_row = false, fast_col = false;
  int* d_list = nullptr;
};

// Size-specialised kernels available for (C, half row length) and (C, n0).
bool has_fast_row(int C, int nh) {
  if (C == 3) return nh == 32 || nh == 64 || nh == 128 || nh == 192 || nh == 256;
  return nh == 32 || nh == 64 || nh == 128;
}
bool has_fast_col(int C, int n0) {
  if (C == 3) return n0 == 64 || n0 == 128 || n0 == 256 || n0 == 384 || n0 == 512;
  return n0 == 64 || n0 == 128;
}
// ------------------------------------------------------------------ kernel variants
// Row-kernel variants per (C, half length): the selected one (default 0) is
// kept per process; mor_tune_set / mor_autotune change it.
std::mutex g_var_mu;
std::map<std::pair<int, int>, int> g_row_var;  // (C, nh) -> variant

template <int C, int NH, int V = 0>
int row_rb_v(int v) {
  if constexpr (V < RowVar<C, NH>::count) {
    return v == V ? RowCfg<C, NH, V>::RB : row_rb_v<C, NH, V + 1>(v);
  } else {
    return -1;
  }
}

int row_variants(int C, int nh) {
  if (C == 3) {
    switch (nh) {
      case 32: return RowVar<3, 32>::count;
      case 64: return RowVar<3, 64>::count;
      case 128: return RowVar<3, 128>::count;
      case 192: return RowVar<3, 192>::count;
      case 256: return RowVar<3, 256>::count;
      default: return 0;
    }
  }
  switch (nh) {
    case 32: return RowVar<6, 32>::count;
    case 64: return RowVar<6, 64>::count;
    case 128: return RowVar<6, 128>::count;
    default: return 0;
  }
}

// Row variant of a size: the tuned one, else the default.  The J2 law holds
// more registers per point (state in, state out), so with J2 phases a size may
// default to a variant with a smaller register pass (measured on the 512^2
// load path: radix-4 register pass, 118 vs 132 ms per path).
int row_variant(int C, int nh, bool j2 = false) {
  std::lock_guard<std::mutex> lk(g_var_mu);
  auto it = g_row_var.find({C, nh});
  if (it != g_row_var.end()) return it->second;
  // with the plastic state in registers the radix-4 register passes keep
  // more waves resident than the defaults (measured on J2 load paths)
  if (j2 && C == 3 && nh == 256) return 4;
  if (j2 && C == 3 && nh == 192) return 2;
  return 0;
}

int fast_rb(int C, int nh, int v) {
  if (C == 3) {
    switch (nh) {
      case 32: return row_rb_v<3, 32>(v);
      case 64: return row_rb_v<3, 64>(v);
      case 128: return row_rb_v<3, 128>(v);
      case 192: return row_rb_v<3, 192>(v);
      default: return row_rb_v<3, 256>(v);
    }
  }
  switch (nh) {
    case 32: return row_rb_v<6, 32>(v);
    case 64: return row_rb_v<6, 64>(v);
    default: return row_rb_v<6, 128>(v);
  }
}
// Column-kernel variants per (C, n0), selected like the row variants.
std::map<std::pair<int, int>, int> g_col_var;  // (C, n0) -> variant

template <int C, int N0, int V = 0>
int col_cb_v(int v) {
  if constexpr (V < ColVar<C, N0>::count) {
    return v == V ? ColCfg<C, N0, V>::CB : col_cb_v<C, N0, V + 1>(v);
  } else {
    return -1;
  }
}

int col_variants(int C, int n0) {
  if (C == 3) {
    switch (n0) {
      case 64: return ColVar<3, 64>::count;
      case 128: return ColVar<3, 128>::count;
      case 256: return ColVar<3, 256>::count;
      case 384: return ColVar<3, 384>::count;
      case 512: return ColVar<3, 512>::count;
      default: return 0;
    }
  }
  switch (n0) {
    case 64: return ColVar<6, 64>::count;
    case 128: return ColVar<6, 128>::count;
    default: return 0;
  }
}

int col_variant(int C, int n0) {
  std::lock_guard<std::mutex> lk(g_var_mu);
  auto it = g_col_var.find({C, n0});
  return it == g_col_var.end() ? 0 : it->second;
}

int fast_cb(int C, int n0, int v) {
  if (C == 3) {
    switch (n0) {
      case 64: return col_cb_v<3, 64>(v);
      case 128: return col_cb_v<3, 128>(v);
      case 256: return col_cb_v<3, 256>(v);
      case 384: return col_cb_v<3, 384>(v);
      default: return col_cb_v<3, 512>(v);
    }
  }
  return n0 == 64 ? col_cb_v<6, 64>(v) : col_cb_v<6, 128>(v);
}

struct SolveCtx {
  hipStream_t st = nullptr;
  Workspace* ws = nullptr;
  int C = 3, S = 4, NST = 5, ndim = 2;
  int64_t B = 0;
  std::vector<Group> groups;
  PlanDev* d_plans = nullptr;
  RveState* d_st = nullptr;
  double* d_ebar = nullptr;
  cpx<float>* d_yl = nullptr;
  cpx<float>* d_yc = nullptr;
  cpx<float>* d_coef = nullptr;
  double* d_part = nullptr;
  double* d_sigpart = nullptr;
  double* d_eff = nullptr;
  unsigned int* d_active = nullptr;
  int* d_nblk = nullptr;
  float* d_jstate = nullptr;
  Offs off{};
  MatDev mat{};
  bool j2 = false;
  std::vector<int64_t> coef_off_h, field_off_h;
  std::vector<int> ncoef_h;
  std::vector<EventPair> events;
  std::vector<std::vector<char>> keep;  // host staging that must outlive async copies
  std::vector<PlanDev> plan_dev;         // plan of every RVE (host copy)
  bool want_eps = false, want_sig = false;
  bool capturing = false;  // kernels are being recorded into a hipGraph: no timing events
  bool dft = false;        // last-axis transform as MFMA GEMMs instead of the row FFT
  int dft_prec = DFT_F32;  // DFT_F32 or DFT_X3 (split bf16)
  float* d_dfte = nullptr; // DFT path: real field per RVE [C][N] (strain, then polarisation)
  bool persist = false;    // persistent schedule of the specialised row/column kernels
  int* d_alist = nullptr;  // [B] active RVEs per group (group segments as in the lists)
  int* d_nact = nullptr;   // [groups] active count per group
  bool fp64 = false;       // FP64 fields and coefficients (generic kernels, Hooke phases)
  MatDev64 mat64{};
  // mor_solve_noalloc: every buffer is carved from the library's fixed
  // device scratch array (no workspace, no events, no pinned memory)
  bool noalloc = false;
  unsigned char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  unsigned int h_active_local = 0;
  size_t pin_used = 0;       // bytes of the workspace's pinned staging taken by this solve
  bool pin_claimed = false;  // the staging was made ready for this solve
  cpx<double>* yl64() const { return reinterpret_cast<cpx<double>*>(d_yl); }
  cpx<double>* yc64() const { return reinterpret_cast<cpx<double>*>(d_yc); }
  cpx<double>* coef64() const { return reinterpret_cast<cpx<double>*>(d_coef); }
};

// A solve buffer: from the per-stream workspace, or carved from the fixed
// scratch array of a no-allocation solve (256-byte aligned pieces).
template <typename T>
mor_status cx_get(SolveCtx& cx, const char* name, size_t count, T** out) {
  if (!cx.noalloc) return cx.ws->get(name, count, out);
  const size_t bytes = (std::max<size_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
  if (bytes > cx.arena_cap - cx.arena_used) {
    mor_set_error(std::string("mor_solve_noalloc: the solve needs more than the ") +
                  std::to_string(cx.arena_cap >> 20) + " MiB scratch array (buffer " + name +
                  "); use fewer RVEs per call");
    return MOR_E_INVALID_ARG;
  }
  *out = reinterpret_cast<T*>(cx.arena + cx.arena_used);
  cx.arena_used += bytes;
  return MOR_OK;
}

__global__ void k_zero_f32(float* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

constexpr size_t kPinStageMax = (size_t)64 << 20;

// nb bytes of the workspace's pinned staging for one transfer of this
// solve, or nullptr (no workspace, or the staging is too small this time).
// Each transfer gets its own range: the solve never reuses one while a copy
// may still read or write it, and the next solve on the stream waits for
// the last copy before it starts over.
unsigned char* pin_slot(SolveCtx& cx, size_t nb) {
  if (!cx.ws) return nullptr;
  Workspace& w = *cx.ws;
  if (!cx.pin_claimed) {
    cx.pin_claimed = true;
    if (w.pin_busy) {
      (void)hipEventSynchronize(w.pin_ev);
      w.pin_busy = false;
    }
    if (w.pin_need > w.pin_cap && w.pin_need <= kPinStageMax) {
      if (w.pin) (void)hipHostFree(w.pin);
      w.pin = nullptr;
      w.pin_cap = 0;
      if (hipHostMalloc((void**)&w.pin, w.pin_need, hipHostMallocDefault) == hipSuccess) {
        w.pin_cap = w.pin_need;
      } else {
        (void)hipGetLastError();
        w.pin = nullptr;
      }
    }
    if (!w.pin_ev && hipEventCreateWithFlags(&w.pin_ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      w.pin_ev = nullptr;
    }
  }
  const size_t off = (cx.pin_used + 255) / 256 * 256;
  cx.pin_used = off + nb;
  w.pin_need = std::max(w.pin_need, cx.pin_used);
  return (w.pin && w.pin_ev && cx.pin_used <= w.pin_cap) ? w.pin + off : nullptr;
}

// The last queued copy through the pinned staging.
mor_status pin_mark(SolveCtx& cx) {
  MOR_HIP_TRY(hipEventRecord(cx.ws->pin_ev, cx.st));
  cx.ws->pin_busy = true;
  return MOR_OK;
}

// Asynchronous upload from pinned staging, else from a host copy kept alive
// until the solve ends.
template <typename T>
mor_status upload(SolveCtx& cx, T* dst, const std::vector<T>& src) {
  if (src.empty()) return MOR_OK;
  const size_t nb = src.size() * sizeof(T);
  if (unsigned char* pin = pin_slot(cx, nb)) {
    std::memcpy(pin, src.data(), nb);
    MOR_HIP_TRY(hipMemcpyAsync(dst, pin, nb, hipMemcpyHostToDevice, cx.st));
    return pin_mark(cx);
  }
  cx.keep.emplace_back(nb);
  std::memcpy(cx.keep.back().data(), src.data(), nb);
  MOR_HIP_TRY(hipMemcpyAsync(dst, cx.keep.back().data(), nb, hipMemcpyHostToDevice, cx.st));
  return MOR_OK;
}

bool finite(double v) { return std::isfinite(v); }

mor_status check_phase(const mor_phase* ph, int ndim) {
  for (int p = 0; p < 2; ++p) {
    const mor_phase& q = ph[p];
    if (!finite(q.lambda) || !finite(q.mu) || !finite(q.sigma_y0) || !finite(q.H)) {
      mor_set_error("phase parameters must be finite");
      return MOR_E_INVALID_ARG;
    }
    if (q.mu <= 0.0) {
      mor_set_error("phase shear modulus must be > 0");
      return MOR_E_INVALID_ARG;
    }
    if ((ndim == 2 && q.lambda + q.mu <= 0.0) || (ndim == 3 && q.lambda + 2.0 * q.mu / 3.0 <= 0.0)) {
      mor_set_error("phase bulk modulus must be > 0");
      return MOR_E_INVALID_ARG;
    }
    if (q.plastic && (q.sigma_y0 <= 0.0 || q.H < 0.0)) {
      mor_set_error("plastic phase needs sigma_y0 > 0 and H >= 0");
      return MOR_E_INVALID_ARG;
    }
  }
  return MOR_OK;
}

MatDev make_mat(const mor_phase* ph) {
  MatDev m{};
  for (int p = 0; p < 2; ++p) {
    m.lam[p] = (float)ph[p].lambda;
    m.mu[p] = (float)ph[p].mu;
    m.sy[p] = (float)ph[p].sigma_y0;
    m.H[p] = (float)ph[p].H;
    m.plastic[p] = ph[p].plastic ? 1 : 0;
  }
  const double lam0 = 0.5 * (ph[0].lambda + ph[1].lambda);
  const double mu0 = 0.5 * (ph[0].mu + ph[1].mu);
  m.lam0 = (float)lam0;
  m.mu0 = (float)mu0;
  for (int p = 0; p < 2; ++p) {
    m.dl[p] = m.lam[p] - m.lam0;
    m.dm[p] = 2.f * (m.mu[p] - m.mu0);
  }
  m.g_inv_mu0 = (float)(1.0 / mu0);
  m.g_k = (float)((lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0)));
  return m;
}


MatDev64 make_mat64(const mor_phase* ph) {
  MatDev64 m{};
  for (int p = 0; p < 2; ++p) {
    m.lam[p] = ph[p].lambda;
    m.mu[p] = ph[p].mu;
  }
  m.lam0 = 0.5 * (ph[0].lambda + ph[1].lambda);
  m.mu0 = 0.5 * (ph[0].mu + ph[1].mu);
  for (int p = 0; p < 2; ++p) {
    m.dl[p] = m.lam[p] - m.lam0;
    m.dm[p] = 2.0 * (m.mu[p] - m.mu0);
  }
  m.g_inv_mu0 = 1.0 / m.mu0;
  m.g_k = (m.lam0 + m.mu0) / (m.mu0 * (m.lam0 + 2.0 * m.mu0));
  return m;
}

void ev_begin(SolveCtx& cx, int kind, hipEvent_t* a) {
  if (!g_prof_on || cx.capturing || cx.noalloc) return;
  *a = cx.ws->event();
  (void)hipEventRecord(*a, cx.st);
  (void)kind;
}
void ev_end(SolveCtx& cx, int kind, hipEvent_t a) {
  if (!g_prof_on || cx.capturing || cx.noalloc) return;
  hipEvent_t b = cx.ws->event();
  (void)hipEventRecord(b, cx.st);
  cx.events.push_back({a, b, kind});
}


// ------------------------------------------------------------------ launches
template <int C, int NH, int V, int MODE, int MAT>
void go_row_fast_v(SolveCtx& cx, Group& g, float* eps, float* sig, int rows) {
  if constexpr (V < RowVar<C, NH>::count) {
    using Cfg = RowCfg<C, NH, V>;
    dim3 gr((rows + Cfg::RB - 1) / Cfg::RB, (unsigned)g.rves.size());
    k_row_fast<C, NH, V, MODE, MAT><<<gr, row_threads<C, NH, V>(), row_lds_bytes<C, NH, V>(), cx.st>>>(
        cx.d_plans, g.d_list, cx.d_st, cx.d_yl, cx.off, cx.mat, cx.d_jstate, eps, sig, cx.d_sigpart);
  }
}

template <int C, int NH, int MODE, int MAT>
void go_row_fast(SolveCtx& cx, Group& g, float* eps, float* sig, int rows) {
  static_assert(RowVar<C, NH>::count <= 11, "dispatch covers eleven variants");
  switch (g.rvar) {
    case 0: go_row_fast_v<C, NH, 0, MODE, MAT>(cx, g, eps, sig, rows); break;
    case 1: go_row_fast_v<C, NH, 1, MODE, MAT>(cx, g, eps, sig, rows); break;
    case 2: go_row_fast_v<C, NH, 2, MODE, MAT>(cx, g, eps, sig, rows); break;
    case 3: go_row_fast_v<C, NH, 3, MODE, MAT>(cx, g, eps, sig, rows); break;
    case 4: go_row_fast_v<C, NH, 4, MODE, MAT>(cx, g, eps, sig, rows); break;
    case 5: go_row_fast_v<C, NH, 5, MODE, MAT>(cx, g, eps, sig, rows); break;
    case 6: go_row_fast_v<C, NH, 6, MODE, MAT>(cx, g, eps, sig, rows); break;
    case 7: go_row_fast_v<C, NH, 7, MODE, MAT>(cx, g, eps, sig, rows); break;
    case 8: go_row_fast_v<C, NH, 8, MODE, MAT>(cx, g, eps, sig, rows); break;
    case 9: go_row_fast_v<C, NH, 9, MODE, MAT>(cx, g, eps, sig, rows); break;
    default: go_row_fast_v<C, NH, 10, MODE, MAT>(cx, g, eps, sig, rows); break;
  }
}

template <int C, int MODE, int MAT>
void row_fast(SolveCtx& cx, Group& g, float* eps, float* sig) {
  const int nlen = C == 3 ? g.n1 : g.n2;
  const int rows = C == 3 ? g.n0 : g.n0 * g.n1;
  if constexpr (C == 3) {
    switch (nlen / 2) {
      case 32: go_row_fast<3, 32, MODE, MAT>(cx, g, eps, sig, rows); break;
      case 64: go_row_fast<3, 64, MODE, MAT>(cx, g, eps, sig, rows); break;
      case 128: go_row_fast<3, 128, MODE, MAT>(cx, g, eps, sig, rows); break;
      case 192: go_row_fast<3, 192, MODE, MAT>(cx, g, eps, sig, rows); break;
      default: go_row_fast<3, 256, MODE, MAT>(cx, g, eps, sig, rows); break;
    }
  } else {
    switch (nlen / 2) {
      case 32: go_row_fast<6, 32, MODE, MAT>(cx, g, eps, sig, rows); break;
      case 64: go_row_fast<6, 64, MODE, MAT>(cx, g, eps, sig, rows); break;
      default: go_row_fast<6, 128, MODE, MAT>(cx, g, eps, sig, rows); break;
    }
  }
}

template <int C, int N0, int V, int MODE>
void go_col_fast_v(SolveCtx& cx, Group& g, const cpx<float>* warm) {
  if constexpr (V < ColVar<C, N0>::count) {
    using Cfg = ColCfg<C, N0, V>;
    dim3 gc((g.ncol_max + Cfg::CB - 1) / Cfg::CB, (unsigned)g.rves.size());
    k_col_fast<C, N0, V, MODE><<<gc, col_threads<C, N0, V>(), col_lds_bytes<C, N0, V>(), cx.st>>>(
        cx.d_plans, g.d_list, cx.d_st, cx.d_ebar, cx.d_yc, cx.d_coef, warm, cx.off, cx.d_part, cx.mat);
  }
}

template <int C, int N0, int MODE>
void go_col_fast(SolveCtx& cx, Group& g, const cpx<float>* warm) {
  static_assert(ColVar<C, N0>::count <= 7, "dispatch covers seven variants");
  switch (g.cvar) {
    case 0: go_col_fast_v<C, N0, 0, MODE>(cx, g, warm); break;
    case 1: go_col_fast_v<C, N0, 1, MODE>(cx, g, warm); break;
    case 2: go_col_fast_v<C, N0, 2, MODE>(cx, g, warm); break;
    case 3: go_col_fast_v<C, N0, 3, MODE>(cx, g, warm); break;
    case 4: go_col_fast_v<C, N0, 4, MODE>(cx, g, warm); break;
    case 5: go_col_fast_v<C, N0, 5, MODE>(cx, g, warm); break;
    default: go_col_fast_v<C, N0, 6, MODE>(cx, g, warm); break;
  }
}

// Persistent grid size: a multiple of the workgroups resident at once on the
// device, capped by the number of items.
int persist_grid(const void* fn, int nt, size_t lds, int64_t items) {
  static std::mutex mu;
  static std::map<const void*, int> cache;
  int per = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(fn);
    if (it != cache.end()) per = it->second;
  }
  if (per == 0) {
    int nb = 0, dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, nt, lds) != hipSuccess || nb < 1) nb = 1;
    // four workgroups per resident slot: the queue keeps the dispatcher fed
    // while workgroups of the previous round drain
    per = std::max(1, 4 * nb * std::max(ncu, 1));
    std::lock_guard<std::mutex> lk(mu);
    cache[fn] = per;
  }
  return (int)std::max<int64_t>(1, std::min<int64_t>(per, items));
}

template <int C, int NH, int V, int MAT>
void go_row_persist_v(SolveCtx& cx, Group& g, int rows) {
  if constexpr (V < RowVar<C, NH>::count) {
    using Cfg = RowCfg<C, NH, V>;
    const int ntiles = (rows + Cfg::RB - 1) / Cfg::RB;
    auto fn = k_row_persist<C, NH, V, MAT>;
    const int grid = persist_grid((const void*)fn, row_threads<C, NH, V>(), row_lds_bytes<C, NH, V>(),
                                  (int64_t)ntiles * g.rves.size());
    fn<<<grid, row_threads<C, NH, V>(), row_lds_bytes<C, NH, V>(), cx.st>>>(
        cx.d_plans, g.d_alist, cx.d_nact + g.gidx, ntiles, cx.d_st, cx.d_yl, cx.off, cx.mat, cx.d_jstate);
  }
}

template <int C, int NH, int MAT>
void go_row_persist(SolveCtx& cx, Group& g, int rows) {
  static_assert(RowVar<C, NH>::count <= 11, "dispatch covers eleven variants");
  switch (g.rvar) {
    case 0: go_row_persist_v<C, NH, 0, MAT>(cx, g, rows); break;
    case 1: go_row_persist_v<C, NH, 1, MAT>(cx, g, rows); break;
    case 2: go_row_persist_v<C, NH, 2, MAT>(cx, g, rows); break;
    case 3: go_row_persist_v<C, NH, 3, MAT>(cx, g, rows); break;
    case 4: go_row_persist_v<C, NH, 4, MAT>(cx, g, rows); break;
    case 5: go_row_persist_v<C, NH, 5, MAT>(cx, g, rows); break;
    case 6: go_row_persist_v<C, NH, 6, MAT>(cx, g, rows); break;
    case 7: go_row_persist_v<C, NH, 7, MAT>(cx, g, rows); break;
    case 8: go_row_persist_v<C, NH, 8, MAT>(cx, g, rows); break;
    case 9: go_row_persist_v<C, NH, 9, MAT>(cx, g, rows); break;
    default: go_row_persist_v<C, NH, 10, MAT>(cx, g, rows); break;
  }
}

template <int C, int MAT>
void row_persist(SolveCtx& cx, Group& g) {
  const int nlen = C == 3 ? g.n1 : g.n2;
  const int rows = C == 3 ? g.n0 : g.n0 * g.n1;
  if constexpr (C == 3) {
    switch (nlen / 2) {
      case 32: go_row_persist<3, 32, MAT>(cx, g, rows); break;
      case 64: go_row_persist<3, 64, MAT>(cx, g, rows); break;
      case 128: go_row_persist<3, 128, MAT>(cx, g, rows); break;
      case 192: go_row_persist<3, 192, MAT>(cx, g, rows); break;
      default: go_row_persist<3, 256, MAT>(cx, g, rows); break;
    }
  } else {
    switch (nlen / 2) {
      case 32: go_row_persist<6, 32, MAT>(cx, g, rows); break;
      case 64: go_row_persist<6, 64, MAT>(cx, g, rows); break;
      default: go_row_persist<6, 128, MAT>(cx, g, rows); break;
    }
  }
}

template <int C, int N0, int V>
void go_col_persist_v(SolveCtx& cx, Group& g) {
  if constexpr (V < ColVar<C, N0>::count) {
    using Cfg = ColCfg<C, N0, V>;
    const int ntiles = (g.ncol_max + Cfg::CB - 1) / Cfg::CB;
    auto fn = k_col_persist<C, N0, V>;
    const int grid = persist_grid((const void*)fn, col_threads<C, N0, V>(), col_lds_bytes<C, N0, V>(),
                                  (int64_t)ntiles * g.rves.size());
    fn<<<grid, col_threads<C, N0, V>(), col_lds_bytes<C, N0, V>(), cx.st>>>(
        cx.d_plans, g.d_alist, cx.d_nact + g.gidx, ntiles, cx.d_st, cx.d_ebar, cx.d_yc, cx.d_coef, cx.off,
        cx.d_part, cx.mat);
  }
}

template <int C, int N0>
void go_col_persist(SolveCtx& cx, Group& g) {
  switch (g.cvar) {
    case 0: go_col_persist_v<C, N0, 0>(cx, g); break;
    case 1: go_col_persist_v<C, N0, 1>(cx, g); break;
    case 2: go_col_persist_v<C, N0, 2>(cx, g); break;
    case 3: go_col_persist_v<C, N0, 3>(cx, g); break;
    case 4: go_col_persist_v<C, N0, 4>(cx, g); break;
    case 5: go_col_persist_v<C, N0, 5>(cx, g); break;
    default: go_col_persist_v<C, N0, 6>(cx, g); break;
  }
}

template <int C>
void col_persist(SolveCtx& cx, Group& g) {
  if constexpr (C == 3) {
    switch (g.n0) {
      case 64: go_col_persist<3, 64>(cx, g); break;
      case 128: go_col_persist<3, 128>(cx, g); break;
      case 256: go_col_persist<3, 256>(cx, g); break;
      case 384: go_col_persist<3, 384>(cx, g); break;
      default: go_col_persist<3, 512>(cx, g); break;
    }
  } else {
    if (g.n0 == 64) go_col_persist<6, 64>(cx, g);
    else go_col_persist<6, 128>(cx, g);
  }
}

// 3D axis-1 transform of a group: specialised kernels for n1 = 32/64/128,
// the generic runtime-radix kernel otherwise.
bool has_fast_mid(int n1) { return n1 == 32 || n1 == 64 || n1 == 128; }

template <int N1, int DIR>
void go_mid_fast(SolveCtx& cx, Group& g, int check_active) {
  dim3 gm(6 * ((g.n0 + MidCfg<N1>::XB - 1) / MidCfg<N1>::XB), g.nlast_max, (unsigned)g.rves.size());
  k_mid_fast<6, N1, DIR><<<gm, mid_threads<N1>(), mid_lds_bytes<N1>(), cx.st>>>(
      cx.d_plans, g.d_list, cx.d_st, cx.d_yl, cx.d_yc, cx.off, check_active);
}

template <int DIR>
void launch_mid(SolveCtx& cx, Group& g, int check_active) {
  if (has_fast_mid(g.n1) && !cx.fp64) {
    switch (g.n1) {
      case 32: go_mid_fast<32, DIR>(cx, g, check_active); break;
      case 64: go_mid_fast<64, DIR>(cx, g, check_active); break;
      default: go_mid_fast<128, DIR>(cx, g, check_active); break;
    }
  } else if (cx.fp64) {
    const size_t shm = (size_t)(g.n1 + 2 * 6 * g.xb * g.n1) * sizeof(cpx<double>);
    dim3 gm((g.n0 + g.xb - 1) / g.xb, g.nlast_max, (unsigned)g.rves.size());
    k_mid<6, DIR, double><<<gm, 256, shm, cx.st>>>(cx.d_plans, g.d_list, cx.d_st, cx.yl64(), cx.yc64(), cx.off,
                                                   g.xb, check_active);
  } else {
    const size_t shm = (size_t)(g.n1 + 2 * 6 * g.xb * g.n1) * sizeof(cpx<float>);
    dim3 gm((g.n0 + g.xb - 1) / g.xb, g.nlast_max, (unsigned)g.rves.size());
    k_mid<6, DIR><<<gm, 256, shm, cx.st>>>(cx.d_plans, g.d_list, cx.d_st, cx.d_yl, cx.d_yc, cx.off, g.xb,
                                           check_active);
  }
}

template <int C, int MODE>
void col_fast(SolveCtx& cx, Group& g, const cpx<float>* warm) {
  if constexpr (C == 3) {
    switch (g.n0) {
      case 64: go_col_fast<3, 64, MODE>(cx, g, warm); break;
      case 128: go_col_fast<3, 128, MODE>(cx, g, warm); break;
      case 256: go_col_fast<3, 256, MODE>(cx, g, warm); break;
      case 384: go_col_fast<3, 384, MODE>(cx, g, warm); break;
      default: go_col_fast<3, 512, MODE>(cx, g, warm); break;
    }
  } else {
    if (g.n0 == 64) go_col_fast<6, 64, MODE>(cx, g, warm);
    else go_col_fast<6, 128, MODE>(cx, g, warm);
  }
}

template <int C>
mor_status launch_init(SolveCtx& cx, Group& g, const cpx<float>* warm) {
  const size_t shc = (size_t)(g.n0 + 2 * C * g.cb * g.n0) * sizeof(cpx<float>);
  dim3 grid((g.ncol_max + g.cb - 1) / g.cb, (unsigned)g.rves.size());
  hipEvent_t a{};
  ev_begin(cx, PK_INIT, &a);
  if (cx.fp64)
    k_col<C, MODE_INIT, double, MatDev64><<<grid, 256, 2 * shc, cx.st>>>(
        cx.d_plans, g.d_list, cx.d_st, cx.d_ebar, cx.yc64(), cx.coef64(), warm, cx.off, cx.d_part, cx.mat64, g.cb);
  else if (g.fast_col)
    col_fast<C, MODE_INIT>(cx, g, warm);
  else
    k_col<C, MODE_INIT><<<grid, 256, shc, cx.st>>>(cx.d_plans, g.d_list, cx.d_st, cx.d_ebar, cx.d_yc, cx.d_coef,
                                                   warm, cx.off, cx.d_part, cx.mat, g.cb);
  MOR_LAUNCH_CHECK("col(init)");
  ev_end(cx, PK_INIT, a);
  if (C == 6) {
    ev_begin(cx, PK_MIDI, &a);
    launch_mid<+1>(cx, g, 0);
    MOR_LAUNCH_CHECK("mid(inv)");
    ev_end(cx, PK_MIDI, a);
  }
  return MOR_OK;
}

// Last-axis stage of an iteration on the DFT path: inverse GEMM, pointwise
// step a), forward GEMM.
constexpr int kDftLmax = 512;
constexpr int kDftRb = 8;  // rows per block of the pointwise kernel

// Workgroup tiles of 128 field rows where every component's rows split
// evenly into them (two 32x32 blocks per wavefront share each twiddle
// fragment), else 64.
template <int PREC>
void dft_inverse(SolveCtx& cx, Group& g, int C, int rows, int L, int mode_iter) {
  if (rows % (2 * DFT_T) == 0) {
    dim3 gi(L / DFT_T, C * rows / (2 * DFT_T), (unsigned)g.rves.size());
    k_dft_inv<PREC, kDftLmax, 2><<<gi, 256, 0, cx.st>>>(cx.d_plans, g.d_list, cx.d_st, cx.d_yl, cx.off, cx.d_dfte,
                                                        C, mode_iter);
  } else {
    dim3 gi(L / DFT_T, C * rows / DFT_T, (unsigned)g.rves.size());
    k_dft_inv<PREC, kDftLmax, 1><<<gi, 256, 0, cx.st>>>(cx.d_plans, g.d_list, cx.d_st, cx.d_yl, cx.off, cx.d_dfte,
                                                        C, mode_iter);
  }
}

template <int PREC>
void dft_forward(SolveCtx& cx, Group& g, int C, int rows) {
  if (rows % (2 * DFT_T) == 0) {
    dim3 gf((2 * g.nlast_max + DFT_T - 1) / DFT_T, C * rows / (2 * DFT_T), (unsigned)g.rves.size());
    k_dft_fwd<PREC, kDftLmax, 2><<<gf, 256, 0, cx.st>>>(cx.d_plans, g.d_list, cx.d_st, cx.d_yl, cx.off, cx.d_dfte,
                                                        C);
  } else {
    dim3 gf((2 * g.nlast_max + DFT_T - 1) / DFT_T, C * rows / DFT_T, (unsigned)g.rves.size());
    k_dft_fwd<PREC, kDftLmax, 1><<<gf, 256, 0, cx.st>>>(cx.d_plans, g.d_list, cx.d_st, cx.d_yl, cx.off, cx.d_dfte,
                                                        C);
  }
}

template <int C, int MAT>
void launch_dft_stage(SolveCtx& cx, Group& g, int rows, int L) {
  if (cx.dft_prec == DFT_X3) dft_inverse<DFT_X3>(cx, g, C, rows, L, 1);
  else dft_inverse<DFT_F32>(cx, g, C, rows, L, 1);
  dim3 gp((rows + kDftRb - 1) / kDftRb, (unsigned)g.rves.size());
  k_dft_point<C, MODE_ITER, MAT><<<gp, 256, 0, cx.st>>>(cx.d_plans, g.d_list, cx.d_st, cx.off, cx.mat, cx.d_dfte,
                                                        cx.d_jstate, nullptr, nullptr, nullptr, kDftRb);
  if (cx.dft_prec == DFT_X3) dft_forward<DFT_X3>(cx, g, C, rows);
  else dft_forward<DFT_F32>(cx, g, C, rows);
}

// Generic row kernel in FP64 (Hooke phases only: setup rejects J2 with FP64,
// and the J2 instantiation reports it rather than launching nothing).
template <int C, int MODE, int MAT>
mor_status launch_row64(SolveCtx& cx, Group& g, dim3 gr, size_t shm, float* eps, float* sig) {
  if constexpr (MAT == MAT_HOOKE) {
    k_row<C, MODE, MAT_HOOKE, double, MatDev64><<<gr, 256, shm, cx.st>>>(
        cx.d_plans, g.d_list, cx.d_st, cx.yl64(), cx.off, cx.mat64, nullptr, eps, sig,
        MODE == MODE_FINAL ? cx.d_sigpart : nullptr, g.rb);
    return MOR_OK;
  } else {
    mor_set_error("MOR_PREC_FP64 supports Hooke phases only (J2 runs in FP32)");
    return MOR_E_UNSUPPORTED;
  }
}

template <int C, int MAT>
mor_status launch_iter(SolveCtx& cx, Group& g) {
  const int nlen = C == 3 ? g.n1 : g.n2;
  const int rows = C == 3 ? g.n0 : g.n0 * g.n1;
  const int nh = nlen / 2;
  const size_t shr = (size_t)(nh + nh + 1 + 2 * C * g.rb * (nh + 1)) * sizeof(cpx<float>);
  dim3 gr((rows + g.rb - 1) / g.rb, (unsigned)g.rves.size());
  hipEvent_t a{};
  const bool pers = cx.persist && !cx.dft;
  if (pers) {
    // queue of this iteration: the group's still-iterating RVEs
    k_active_list<<<1, 1024, 0, cx.st>>>(g.d_list, (int)g.rves.size(), cx.d_st, g.d_alist, cx.d_nact + g.gidx);
    MOR_LAUNCH_CHECK("active_list");
  }
  ev_begin(cx, PK_ROW, &a);
  if (cx.dft)
    launch_dft_stage<C, MAT>(cx, g, rows, nlen);
  else if (cx.fp64) {
    const mor_status s64 = launch_row64<C, MODE_ITER, MAT>(cx, g, gr, 2 * shr, nullptr, nullptr);
    if (s64 != MOR_OK) return s64;
  } else if (g.fast_row && pers)
    row_persist<C, MAT>(cx, g);
  else if (g.fast_row)
    row_fast<C, MODE_ITER, MAT>(cx, g, nullptr, nullptr);
  else
    k_row<C, MODE_ITER, MAT><<<gr, 256, shr, cx.st>>>(cx.d_plans, g.d_list, cx.d_st, cx.d_yl, cx.off, cx.mat,
                                                      cx.d_jstate, nullptr, nullptr, nullptr, g.rb);
  MOR_LAUNCH_CHECK("row");
  ev_end(cx, PK_ROW, a);
  if (C == 6) {
    ev_begin(cx, PK_MIDF, &a);
    launch_mid<-1>(cx, g, 1);
    MOR_LAUNCH_CHECK("mid(fwd)");
    ev_end(cx, PK_MIDF, a);
  }
  const size_t shc = (size_t)(g.n0 + 2 * C * g.cb * g.n0) * sizeof(cpx<float>);
  dim3 gc((g.ncol_max + g.cb - 1) / g.cb, (unsigned)g.rves.size());
  ev_begin(cx, PK_COL, &a);
  if (cx.fp64)
    k_col<C, MODE_ITER, double, MatDev64><<<gc, 256, 2 * shc, cx.st>>>(
        cx.d_plans, g.d_list, cx.d_st, cx.d_ebar, cx.yc64(), cx.coef64(), nullptr, cx.off, cx.d_part, cx.mat64, g.cb);
  else if (g.fast_col && pers)
    col_persist<C>(cx, g);
  else if (g.fast_col)
    col_fast<C, MODE_ITER>(cx, g, nullptr);
  else
    k_col<C, MODE_ITER><<<gc, 256, shc, cx.st>>>(cx.d_plans, g.d_list, cx.d_st, cx.d_ebar, cx.d_yc, cx.d_coef,
                                                 nullptr, cx.off, cx.d_part, cx.mat, g.cb);
  MOR_LAUNCH_CHECK("col");
  ev_end(cx, PK_COL, a);
  if (C == 6) {
    ev_begin(cx, PK_MIDI, &a);
    launch_mid<+1>(cx, g, 1);
    MOR_LAUNCH_CHECK("mid(inv)");
    ev_end(cx, PK_MIDI, a);
  }
  // the stop decision comes last: every stage of this iteration has run
  const int nrv = (int)g.rves.size();
  k_converge<<<(nrv + kConvergeRvesPerBlock - 1) / kConvergeRvesPerBlock, 256, 0, cx.st>>>(
      cx.d_plans, g.d_list, nrv, cx.d_st, cx.d_part, cx.off, g.cb, cx.d_active);
  MOR_LAUNCH_CHECK("converge");
  return MOR_OK;
}

template <int C, int MAT>
mor_status launch_final(SolveCtx& cx, Group& g, float* eps, float* sig) {
  const int nlen = C == 3 ? g.n1 : g.n2;
  const int rows = C == 3 ? g.n0 : g.n0 * g.n1;
  const int nh = nlen / 2;
  const size_t shr = (size_t)(nh + nh + 1 + 2 * C * g.rb * (nh + 1)) * sizeof(cpx<float>);
  dim3 gr((rows + g.rb - 1) / g.rb, (unsigned)g.rves.size());
  hipEvent_t a{};
  ev_begin(cx, PK_FINAL, &a);
  if (cx.dft) {
    if (cx.dft_prec == DFT_X3) dft_inverse<DFT_X3>(cx, g, C, rows, nlen, 0);
    else dft_inverse<DFT_F32>(cx, g, C, rows, nlen, 0);
    dim3 gp((rows + kDftRb - 1) / kDftRb, (unsigned)g.rves.size());
    k_dft_point<C, MODE_FINAL, MAT><<<gp, 256, 0, cx.st>>>(cx.d_plans, g.d_list, cx.d_st, cx.off, cx.mat, cx.d_dfte,
                                                           cx.d_jstate, eps, sig, cx.d_sigpart, kDftRb);
  } else if (cx.fp64) {
    const mor_status s64 = launch_row64<C, MODE_FINAL, MAT>(cx, g, gr, 2 * shr, eps, sig);
    if (s64 != MOR_OK) return s64;
  } else if (g.fast_row)
    row_fast<C, MODE_FINAL, MAT>(cx, g, eps, sig);
  else
    k_row<C, MODE_FINAL, MAT><<<gr, 256, shr, cx.st>>>(cx.d_plans, g.d_list, cx.d_st, cx.d_yl, cx.off, cx.mat,
                                                       cx.d_jstate, eps, sig, cx.d_sigpart, g.rb);
  MOR_LAUNCH_CHECK("row(final)");
  ev_end(cx, PK_FINAL, a);
  constexpr int S = Comp<C>::S;
  const int n = (int)g.rves.size() * S;  // one wavefront each
  k_sig_reduce<S><<<(n + 3) / 4, 256, 0, cx.st>>>(cx.d_plans, cx.d_st, g.d_list, (int)g.rves.size(), cx.d_sigpart, cx.off,
                                                      cx.d_nblk, cx.d_eff, S);
  MOR_LAUNCH_CHECK("sig_reduce");
  return MOR_OK;
}

mor_status do_init(SolveCtx& cx, Group& g, const cpx<float>* warm) {
  return cx.C == 3 ? launch_init<3>(cx, g, warm) : launch_init<6>(cx, g, warm);
}
mor_status do_iter(SolveCtx& cx, Group& g) {
  if (cx.C == 3) return cx.j2 ? launch_iter<3, MAT_J2>(cx, g) : launch_iter<3, MAT_HOOKE>(cx, g);
  return cx.j2 ? launch_iter<6, MAT_J2>(cx, g) : launch_iter<6, MAT_HOOKE>(cx, g);
}
mor_status do_final(SolveCtx& cx, Group& g, float* eps, float* sig) {
  if (cx.C == 3) return cx.j2 ? launch_final<3, MAT_J2>(cx, g, eps, sig) : launch_final<3, MAT_HOOKE>(cx, g, eps, sig);
  return cx.j2 ? launch_final<6, MAT_J2>(cx, g, eps, sig) : launch_final<6, MAT_HOOKE>(cx, g, eps, sig);
}

// Per-RVE states for the start of a load step: active, no iterations, the
// residual denominator of that step's macro strain.
std::vector<RveState> fresh_states(const SolveCtx& cx, const std::vector<mor_plan*>& plans,
                                   const std::vector<int>& plan_of, const double* ebar, double tol, int max_iter) {
  std::vector<RveState> hs(cx.B);
  for (int64_t b = 0; b < cx.B; ++b) {
    double nrm2 = 0.0;
    for (int c = 0; c < cx.C; ++c) {
      const double v = ebar[b * cx.C + c];
      nrm2 += (c < (cx.C == 3 ? 2 : 3) ? 1.0 : 2.0) * v * v;
    }
    RveState& r = hs[b];
    r.active = 1;
    r.iters = 0;
    r.status = MOR_OK;
    r.plan = plan_of[b];
    r.resid = 0.0;
    r.denom = (double)plans[plan_of[b]]->N * (nrm2 > 0.0 ? std::sqrt(nrm2) : 1.0);
    r.tol = tol;
    r.max_iter = max_iter;
    r.warm_ok = 1;
  }
  return hs;
}

// Working-set limit of one sub-batch (bytes of transform lines): MI355X's
// 256 MB Infinity Cache less room for the coefficients, tables and phase
// maps the passes also stream.  MOR_SUBBATCH_MIB in the environment sets the
// start value, mor_tune_subbatch changes it (0: one sub-batch per grid).
std::atomic<int64_t>& subbatch_limit() {
  static std::atomic<int64_t> v{[] {
    if (const char* e = getenv("MOR_SUBBATCH_MIB")) {
      char* end = nullptr;
      const long long m = strtoll(e, &end, 10);
      if (end != e && m >= 0 && m < (1LL << 40)) return (int64_t)m << 20;
    }
    return (int64_t)192 << 20;
  }()};
  return v;
}
size_t subbatch_bytes() { return (size_t)subbatch_limit().load(); }
// Fewest RVEs of a sub-batch: below this the per-launch cost of the extra
// launches outweighs the cache hits (3D RVEs of 128^3 lose 3 % when cut into
// runs of two).
std::atomic<int64_t>& subbatch_min_rves() {
  static std::atomic<int64_t> v{128};
  return v;
}

// Prepare the context: plan table, groups, offsets, states.
mor_status setup(SolveCtx& cx, const std::vector<mor_plan*>& plans, const std::vector<int>& plan_of,
                 const double* ebar, int64_t B, const mor_phase* phase, double tol, const mor_solve_opts* opts,
                 float* jstate_user) {
  cx.st = opts ? (hipStream_t)opts->stream : nullptr;
  cx.ws = cx.noalloc ? nullptr : workspace_for(cx.st);
  cx.B = B;
  cx.ndim = plans[0]->ndim;
  cx.C = cx.ndim == 2 ? 3 : 6;
  cx.S = cx.ndim == 2 ? 4 : 6;
  cx.NST = cx.ndim == 2 ? 5 : 7;
  cx.mat = make_mat(phase);
  cx.j2 = phase[0].plastic || phase[1].plastic;
  cx.fp64 = opts && opts->precision == MOR_PREC_FP64;
  if (cx.fp64) {
    cx.mat64 = make_mat64(phase);
    if (cx.j2) {
      mor_set_error("MOR_PREC_FP64 supports Hooke phases only (J2 runs in FP32)");
      return MOR_E_UNSUPPORTED;
    }
    if (opts->transform == MOR_TRANSFORM_DFT) {
      mor_set_error("MOR_PREC_FP64 uses the FFT transform (MOR_TRANSFORM_AUTO or MOR_TRANSFORM_FFT)");
      return MOR_E_UNSUPPORTED;
    }
    if (opts->schedule == MOR_SCHED_PERSISTENT) {
      mor_set_error("MOR_PREC_FP64 runs on the grid schedule only");
      return MOR_E_UNSUPPORTED;
    }
  }
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 10000;
  mor_status s;
  // plan table
  std::vector<PlanDev> pd(plans.size());
  for (size_t i = 0; i < plans.size(); ++i) pd[i] = plans[i]->dev;
  cx.plan_dev.resize(B);
  for (int64_t b = 0; b < B; ++b) cx.plan_dev[b] = plans[plan_of[b]]->dev;
  if ((s = cx_get(cx, "plans", pd.size(), &cx.d_plans)) != MOR_OK) return s;
  if ((s = upload(cx, cx.d_plans, pd)) != MOR_OK) return s;
  // groups by grid
  std::map<std::vector<int>, int> gidx;
  for (int64_t b = 0; b < B; ++b) {
    const mor_plan* p = plans[plan_of[b]];
    std::vector<int> key = {p->ndim, p->n[0], p->n[1], p->n[2]};
    auto it = gidx.find(key);
    int gi;
    if (it == gidx.end()) {
      gi = (int)cx.groups.size();
      gidx[key] = gi;
      Group g;
      g.ndim = p->ndim;
      g.n0 = p->n[0];
      g.n1 = p->n[1];
      g.n2 = p->ndim == 3 ? p->n[2] : 1;
      cx.groups.push_back(g);
    } else {
      gi = it->second;
    }
    Group& g = cx.groups[gi];
    g.rves.push_back((int)b);
    g.ncol_max = std::max(g.ncol_max, p->dev.ncol);
    g.nlast_max = std::max(g.nlast_max, p->dev.nlast);
  }
  // offsets
  std::vector<int64_t> offs(5 * B);
  std::vector<int> nblk(B);
  int64_t yl = 0, yc = 0, co = 0, fo = 0, pa = 0;
  cx.coef_off_h.resize(B);
  cx.field_off_h.resize(B);
  cx.ncoef_h.resize(B);
  // transform of the last axis: the row FFT (default, and AUTO: measured
  // faster on every size), or the MFMA partial DFT
  cx.persist = opts && opts->schedule == MOR_SCHED_PERSISTENT;
  if (opts && (opts->transform == MOR_TRANSFORM_DFT || opts->precision == MOR_PREC_BF16X3)) {
    cx.dft = true;
    cx.dft_prec = opts->precision == MOR_PREC_BF16X3 ? DFT_X3 : DFT_F32;
  }
  for (auto& g : cx.groups) {
    const int nlen = g.ndim == 2 ? g.n1 : g.n2;
    const int rows = g.ndim == 2 ? g.n0 : g.n0 * g.n1;
    if (cx.dft && (rows % DFT_T != 0 || nlen % DFT_T != 0 || nlen > kDftLmax)) {
      mor_set_error("the DFT transform needs rows and last-axis length multiples of 64 (length <= 512)");
      return MOR_E_UNSUPPORTED;
    }
    g.fast_row = !cx.fp64 && has_fast_row(cx.C, nlen / 2);
    g.fast_col = !cx.fp64 && has_fast_col(cx.C, g.n0);
    const int es = cx.fp64 ? (int)sizeof(cpx<double>) : (int)sizeof(cpx<float>);
    if (cx.dft) {
      g.rb = kDftRb;
    } else if (g.fast_row) {
      g.rvar = std::min(row_variant(cx.C, nlen / 2, cx.j2), row_variants(cx.C, nlen / 2) - 1);
      g.rb = fast_rb(cx.C, nlen / 2, g.rvar);
    } else {
      g.rb = rows_per_block(cx.C, nlen, es);
    }
    if (g.fast_col) {
      g.cvar = std::min(col_variant(cx.C, g.n0), col_variants(cx.C, g.n0) - 1);
      g.cb = fast_cb(cx.C, g.n0, g.cvar);
    } else {
      g.cb = cols_per_block(cx.C, g.n0, es);
    }
    g.xb = g.ndim == 3 ? cols_per_block(cx.C, g.n1, es) : 1;
    if (!g.fast_row && !cx.dft) g.rb = std::min(g.rb, rows);
  }
  // Sub-batches: a group's RVEs are cut into runs whose transform lines fit
  // in the device's last-level cache, and the iteration loop runs the chunk
  // of iterations of one sub-batch before the next, so the lines the row
  // pass writes are still cached when the column pass reads them and vice
  // versa (a batch of 1024 256^2 RVEs streams 350 MB of lines per pass).
  {
    const size_t limit = subbatch_bytes();
    const size_t es = cx.fp64 ? sizeof(cpx<double>) : sizeof(cpx<float>);
    std::vector<Group> split;
    for (const Group& g : cx.groups) {
      std::vector<size_t> yb(g.rves.size());
      size_t total = 0;
      for (size_t q = 0; q < g.rves.size(); ++q) {
        const mor_plan* p = plans[plan_of[g.rves[q]]];
        yb[q] = (size_t)cx.C * p->dev.nlast * p->dev.rows * es;
        if (cx.ndim == 3) yb[q] += (size_t)cx.C * p->dev.ncol * p->n[0] * es;
        total += yb[q];
      }
      // as few sub-batches as the limit allows, of about equal size (cut
      // where the running sum passes the next multiple of total / parts)
      const size_t minr = (size_t)std::max<int64_t>(1, subbatch_min_rves().load());
      const size_t parts = limit > 0 ? std::max<size_t>(1, std::min((total + limit - 1) / limit,
                                                                    g.rves.size() / minr))
                                     : 1;
      Group cur = g;
      cur.rves.clear();
      size_t run = 0, cut = 1;
      for (size_t q = 0; q < g.rves.size(); ++q) {
        if (cut < parts && !cur.rves.empty() && (long double)run >= (long double)total * cut / parts) {
          split.push_back(cur);
          cur.rves.clear();
          ++cut;
        }
        cur.rves.push_back(g.rves[q]);
        run += yb[q];
      }
      split.push_back(cur);
    }
    cx.groups.swap(split);
  }
  std::vector<int> gof(B);
  for (size_t gi = 0; gi < cx.groups.size(); ++gi)
    for (int b : cx.groups[gi].rves) gof[b] = (int)gi;
  for (int64_t b = 0; b < B; ++b) {
    const mor_plan* p = plans[plan_of[b]];
    const Group& g = cx.groups[gof[b]];
    const int rows = p->dev.rows;
    offs[0 * B + b] = yl;
    yl += (int64_t)cx.C * p->dev.nlast * rows;
    if (cx.ndim == 3) {
      offs[1 * B + b] = yc;
      yc += (int64_t)cx.C * p->dev.ncol * p->n[0];
    } else {
      offs[1 * B + b] = offs[0 * B + b];
    }
    offs[2 * B + b] = co;
    cx.coef_off_h[b] = co;
    cx.ncoef_h[b] = p->dev.ncoef;
    co += (int64_t)cx.C * p->dev.ncoef;
    offs[3 * B + b] = fo;
    cx.field_off_h[b] = fo;
    fo += p->N;
    offs[4 * B + b] = pa;
    const int nrb = (rows + g.rb - 1) / g.rb;
    const int ncb = (p->dev.ncol + g.cb - 1) / g.cb;
    pa += std::max(nrb, ncb);
    nblk[b] = nrb;
  }
  int64_t* d_offs;
  if ((s = cx_get(cx, "offs", offs.size(), &d_offs)) != MOR_OK) return s;
  if ((s = upload(cx, d_offs, offs)) != MOR_OK) return s;
  cx.off.yl = d_offs;
  cx.off.yc = d_offs + B;
  cx.off.coef = d_offs + 2 * B;
  cx.off.field = d_offs + 3 * B;
  cx.off.part = d_offs + 4 * B;
  // counts in FP32 complex elements; FP64 complex takes two
  const size_t ew = cx.fp64 ? 2 : 1;
  if ((s = cx_get(cx, "yl", (size_t)yl * ew, &cx.d_yl)) != MOR_OK) return s;
  if (cx.ndim == 3) {
    if ((s = cx_get(cx, "yc", (size_t)yc * ew, &cx.d_yc)) != MOR_OK) return s;
  } else {
    cx.d_yc = cx.d_yl;
  }
  if ((s = cx_get(cx, "coef", (size_t)co * ew, &cx.d_coef)) != MOR_OK) return s;
  if (cx.dft && (s = cx_get(cx, "dfte", (size_t)fo * cx.C, &cx.d_dfte)) != MOR_OK) return s;
  if ((s = cx_get(cx, "part", (size_t)pa, &cx.d_part)) != MOR_OK) return s;
  if ((s = cx_get(cx, "sigpart", (size_t)pa * cx.S, &cx.d_sigpart)) != MOR_OK) return s;
  if ((s = cx_get(cx, "eff", (size_t)B * cx.S, &cx.d_eff)) != MOR_OK) return s;
  if ((s = cx_get(cx, "active", 1, &cx.d_active)) != MOR_OK) return s;
  if ((s = cx_get(cx, "ebar", (size_t)B * cx.C, &cx.d_ebar)) != MOR_OK) return s;
  if ((s = cx_get(cx, "state", (size_t)B, &cx.d_st)) != MOR_OK) return s;
  // group lists and final block counts (per group position)
  std::vector<int> lists, nblk_list;
  std::vector<size_t> lstart;
  for (auto& g : cx.groups) {
    lstart.push_back(lists.size());
    for (int b : g.rves) {
      lists.push_back(b);
      nblk_list.push_back(nblk[b]);
    }
  }
  int* d_lists;
  if ((s = cx_get(cx, "lists", lists.size(), &d_lists)) != MOR_OK) return s;
  if ((s = cx_get(cx, "nblk", nblk_list.size(), &cx.d_nblk)) != MOR_OK) return s;
  if ((s = upload(cx, d_lists, lists)) != MOR_OK) return s;
  if ((s = upload(cx, cx.d_nblk, nblk_list)) != MOR_OK) return s;
  for (size_t gi = 0; gi < cx.groups.size(); ++gi) cx.groups[gi].d_list = d_lists + lstart[gi];
  if (cx.persist) {
    if ((s = cx_get(cx, "alist", lists.size(), &cx.d_alist)) != MOR_OK) return s;
    if ((s = cx_get(cx, "nact", cx.groups.size(), &cx.d_nact)) != MOR_OK) return s;
    for (size_t gi = 0; gi < cx.groups.size(); ++gi) {
      cx.groups[gi].gidx = (int)gi;
      cx.groups[gi].d_alist = cx.d_alist + lstart[gi];
    }
  }
  // nblk is indexed by group position in k_sig_reduce: shift per group
  // (k_sig_reduce receives the group's list; its nblk pointer is offset below)
  // states
  std::vector<RveState> hs = fresh_states(cx, plans, plan_of, ebar, tol, max_iter);
  std::vector<double> eb(ebar, ebar + B * cx.C);
  if ((s = upload(cx, cx.d_st, hs)) != MOR_OK) return s;
  if ((s = upload(cx, cx.d_ebar, eb)) != MOR_OK) return s;
  std::vector<unsigned int> act(1, (unsigned int)B);
  if ((s = upload(cx, cx.d_active, act)) != MOR_OK) return s;
  // J2 state
  if (cx.j2) {
    if (jstate_user) {
      cx.d_jstate = jstate_user;
    } else {
      if ((s = cx_get(cx, "jstate", (size_t)fo * cx.NST, &cx.d_jstate)) != MOR_OK) return s;
      if (cx.noalloc) {
        // the scratch array keeps the previous call's contents: a fill kernel
        // (no memset node for callers that capture the solve into a graph)
        k_zero_f32<<<1024, 256, 0, cx.st>>>(cx.d_jstate, (int64_t)fo * cx.NST);
        MOR_LAUNCH_CHECK("zero J2 state");
      } else {
        MOR_HIP_TRY(hipMemsetAsync(cx.d_jstate, 0, (size_t)fo * cx.NST * sizeof(float), cx.st));
      }
    }
  }
  return MOR_OK;
}

// One captured chunk of iterations (owns the graph and its executable).
struct GraphChunk {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~GraphChunk() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
  mor_status record(SolveCtx& cx, int check) {
    hipStream_t solve_st = cx.st;
    cx.st = cx.ws->capture_stream();
    cx.capturing = true;
    mor_status s = MOR_OK;
    hipError_t e = hipStreamBeginCapture(cx.st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      for (auto& g : cx.groups)
        for (int k = 0; k < check && s == MOR_OK; ++k)
          if ((s = do_iter(cx, g)) != MOR_OK) break;
      hipError_t e2 = hipStreamEndCapture(cx.st, &graph);
      if (e2 != hipSuccess && s == MOR_OK) e = e2;
    }
    cx.st = solve_st;
    cx.capturing = false;
    if (s != MOR_OK) return s;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      mor_set_error(std::string("hipGraph capture of the iteration chunk failed: ") + hipGetErrorString(e));
      return MOR_E_DEVICE;
    }
    return MOR_OK;
  }
};

mor_status run(SolveCtx& cx, const cpx<float>* warm, const mor_solve_opts* opts, float* eps, float* sig) {
  mor_status s;
  if (warm) {
    // an RVE whose warm coefficients hold a NaN/Inf starts cold instead
    for (auto& g : cx.groups) {
      k_warm_check<<<(unsigned)g.rves.size(), 256, 0, cx.st>>>(cx.d_plans, g.d_list, (int)g.rves.size(), cx.d_st,
                                                               warm, cx.off, cx.C);
      MOR_LAUNCH_CHECK("warm_check");
    }
  }
  for (auto& g : cx.groups)
    if ((s = do_init(cx, g, warm)) != MOR_OK) return s;
  const int check = (opts && opts->check_every > 0) ? opts->check_every : 8;
  int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 10000;
  int done = 0;
  // With use_graph, one chunk of `check` iterations over all groups is
  // recorded once (on a private stream: capture only records) and replayed
  // as a single graph launch per chunk on the solve stream.  Every launch of
  // a chunk has the same arguments (the iteration state lives in device
  // memory), so the replays are the eager sequence.
  GraphChunk gc;
  if (opts && opts->use_graph) {
    if ((s = gc.record(cx, check)) != MOR_OK) return s;
  }
  while (true) {
    if (gc.exec) {
      MOR_HIP_TRY(hipGraphLaunch(gc.exec, cx.st));
    } else {
      // sub-batch outermost: its lines stay cached across its iterations
      for (auto& g : cx.groups)
        for (int k = 0; k < check; ++k)
          if ((s = do_iter(cx, g)) != MOR_OK) return s;
    }
    done += check;
    unsigned int* hact = cx.noalloc ? &cx.h_active_local : cx.ws->h_active;
    MOR_HIP_TRY(hipMemcpyAsync(hact, cx.d_active, sizeof(unsigned int), hipMemcpyDeviceToHost, cx.st));
    MOR_HIP_TRY(hipStreamSynchronize(cx.st));
    if (*hact == 0u) break;
    if (done > max_iter + check) {
      mor_set_error("iteration loop did not drain");
      return MOR_E_DEVICE;
    }
  }
  // finalize; the nblk pointer is offset per group
  size_t pos = 0;
  int* nblk_base = cx.d_nblk;
  for (auto& g : cx.groups) {
    cx.d_nblk = nblk_base + pos;
    int64_t foff = 0;
    (void)foff;
    if ((s = do_final(cx, g, eps, sig)) != MOR_OK) {
      cx.d_nblk = nblk_base;
      return s;
    }
    pos += g.rves.size();
  }
  cx.d_nblk = nblk_base;
  return MOR_OK;
}

// FP64 coefficients rounded to the FP32 output layout.
__global__ void k_round_c64(const cpx<double>* __restrict__ a, cpx<float>* __restrict__ o, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = {(float)a[i].x, (float)a[i].y};
}

void account(SolveCtx& cx, const std::vector<RveState>& hs, int passes = 1);

mor_status collect(SolveCtx& cx, mor_outputs* out, int eff_stride, std::vector<RveState>* states_out) {
  std::vector<RveState> hs(cx.B);
  std::vector<double> eff((size_t)cx.B * cx.S);
  const size_t hs_nb = hs.size() * sizeof(RveState), eff_nb = eff.size() * sizeof(double);
  unsigned char* hs_pin = pin_slot(cx, hs_nb);
  unsigned char* eff_pin = (out && out->eff_stress) ? pin_slot(cx, eff_nb) : nullptr;
  MOR_HIP_TRY(hipMemcpyAsync(hs_pin ? (void*)hs_pin : (void*)hs.data(), cx.d_st, hs_nb, hipMemcpyDeviceToHost,
                             cx.st));
  if (out && out->eff_stress)
    MOR_HIP_TRY(hipMemcpyAsync(eff_pin ? (void*)eff_pin : (void*)eff.data(), cx.d_eff, eff_nb,
                               hipMemcpyDeviceToHost, cx.st));
  if (hs_pin || eff_pin) {
    mor_status ms = pin_mark(cx);
    if (ms != MOR_OK) return ms;
  }
  if (out && out->coeffs) {
    int64_t tot = 0;
    for (int64_t b = 0; b < cx.B; ++b) tot += (int64_t)cx.C * cx.ncoef_h[b];
    if (cx.fp64) {
      if (tot > 0) {
        k_round_c64<<<(unsigned)((tot + 255) / 256), 256, 0, cx.st>>>(cx.coef64(), (cpx<float>*)out->coeffs, tot);
        MOR_LAUNCH_CHECK("round coefficients");
      }
    } else {
      MOR_HIP_TRY(hipMemcpyAsync(out->coeffs, cx.d_coef, tot * sizeof(cpx<float>), hipMemcpyDeviceToDevice, cx.st));
    }
  }
  MOR_HIP_TRY(hipStreamSynchronize(cx.st));
  if (cx.ws) cx.ws->pin_busy = false;
  if (hs_pin) std::memcpy(hs.data(), hs_pin, hs_nb);
  if (eff_pin) std::memcpy(eff.data(), eff_pin, eff_nb);
  account(cx, hs);
  mor_status worst = MOR_OK;
  for (int64_t b = 0; b < cx.B; ++b) {
    if (out && out->iterations) out->iterations[b] = hs[b].iters;
    if (out && out->residual) out->residual[b] = hs[b].resid;
    if (out && out->eff_stress)
      for (int s = 0; s < cx.S; ++s) out->eff_stress[b * eff_stride + s] = eff[b * cx.S + s];
    if (hs[b].status == MOR_E_NONFINITE) worst = MOR_E_NONFINITE;
    else if (hs[b].status == MOR_E_NOT_CONVERGED && worst == MOR_OK) worst = MOR_E_NOT_CONVERGED;
  }
  if (states_out) *states_out = hs;
  if (worst == MOR_E_NONFINITE) mor_set_error("non-finite residual in at least one RVE");
  if (worst == MOR_E_NOT_CONVERGED) mor_set_error("max_iter reached before tol in at least one RVE");
  return worst;
}

// Per-kernel profile of the work of one solve (or one load step): event
// times of the launches recorded so far, algorithmic bytes from the RVEs'
// iteration counts.  Clears the recorded events.
void account(SolveCtx& cx, const std::vector<RveState>& hs, int passes) {
  if (g_prof_on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& e : cx.events) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
        g_prof[e.kind].ms += ms;
        g_prof[e.kind].launches += 1;
      }
    }
    // Algorithmic HBM bytes of the work done: RVE b ran its row/column (and
    // axis-1) kernels once per iteration, init and final once.
    for (int64_t b = 0; b < cx.B; ++b) {
      const PlanDev& d = cx.plan_dev[b];
      const double it = hs[b].iters;
      const double C = cx.C, L = d.nlen;
      const double ew = cx.fp64 ? 2.0 : 1.0;  // complex elements of FP64 take twice the bytes
      double row = d.rows * (16.0 * ew * C * d.nlast + L);
      // DFT path: spectra in/out plus the real field written, read,
      // rewritten and read again between the GEMMs
      if (cx.dft) row += 16.0 * C * d.N;
      if (cx.j2) row += d.rows * L * 4.0 * cx.NST;
      const double col = d.ncol * 16.0 * ew * C * d.n0 + d.ncoef * (16.0 * ew * C + 17.0);
      const double mid = cx.ndim == 3 ? d.n0 * 8.0 * ew * C * ((double)d.nlast * d.n1 + d.ncol) : 0.0;
      double fin = d.rows * (8.0 * ew * C * d.nlast + L);
      if (cx.dft) fin += 8.0 * C * d.N;
      if (cx.want_eps) fin += (double)d.N * 4.0 * C;
      if (cx.want_sig) fin += (double)d.N * 4.0 * cx.S;
      if (cx.j2) fin += (double)d.N * 8.0 * cx.NST;
      g_prof[PK_ROW].items += (int64_t)it;
      g_prof[PK_ROW].bytes += it * row;
      g_prof[PK_COL].items += (int64_t)it;
      g_prof[PK_COL].bytes += it * col;
      if (cx.ndim == 3) {
        g_prof[PK_MIDF].items += (int64_t)it;
        g_prof[PK_MIDF].bytes += it * mid;
        g_prof[PK_MIDI].items += (int64_t)it + 1;
        g_prof[PK_MIDI].bytes += (it + 1.0) * mid;
      }
      g_prof[PK_FINAL].items += passes;
      g_prof[PK_FINAL].bytes += passes * fin;
      g_prof[PK_INIT].items += passes;
      g_prof[PK_INIT].bytes += passes * (d.ncol * 8.0 * ew * C * d.n0 + d.ncoef * (8.0 * ew + 17.0));
    }
  }
  cx.events.clear();
  if (cx.ws) cx.ws->evnext = 0;
}

mor_status check_common(const double* ebar, int64_t B, int C, const mor_phase* phase, double tol,
                        const mor_solve_opts* opts, int ndim) {
  if (!ebar || !phase) {
    mor_set_error("NULL macro strain or phase");
    return MOR_E_INVALID_ARG;
  }
  if (B < 1) {
    mor_set_error("B must be >= 1");
    return MOR_E_INVALID_ARG;
  }
  if (!(tol > 0.0) || !std::isfinite(tol)) {
    mor_set_error("tol must be a finite number > 0");
    return MOR_E_INVALID_ARG;
  }
  for (int64_t i = 0; i < B * C; ++i)
    if (!std::isfinite(ebar[i])) {
      mor_set_error("macro strain must be finite");
      return MOR_E_INVALID_ARG;
    }
  mor_status s = check_phase(phase, ndim);
  if (s != MOR_OK) return s;
  if (opts) {
    if (opts->max_iter < 0 || opts->check_every < 0) {
      mor_set_error("max_iter and check_every must be >= 0");
      return MOR_E_INVALID_ARG;
    }
    if (opts->precision != MOR_PREC_FP32 && opts->precision != MOR_PREC_BF16X3 &&
        opts->precision != MOR_PREC_FP64) {
      mor_set_error("precision must be MOR_PREC_FP32, MOR_PREC_BF16X3 or MOR_PREC_FP64");
      return MOR_E_INVALID_ARG;
    }
    if (opts->transform < MOR_TRANSFORM_AUTO || opts->transform > MOR_TRANSFORM_DFT) {
      mor_set_error("unknown transform");
      return MOR_E_INVALID_ARG;
    }
    if (opts->schedule != MOR_SCHED_GRID && opts->schedule != MOR_SCHED_PERSISTENT) {
      mor_set_error("unknown schedule");
      return MOR_E_INVALID_ARG;
    }
    if (opts->precision == MOR_PREC_BF16X3 && opts->transform == MOR_TRANSFORM_FFT) {
      mor_set_error("MOR_PREC_BF16X3 applies to the DFT transform only");
      return MOR_E_UNSUPPORTED;
    }
  }
  return MOR_OK;
}

// One solve at a time per stream (the stream's workspace is shared);
// recursive so that a call may hold it around the solves it makes.
std::recursive_mutex& stream_mutex(void* stream) {
  static std::mutex mu;
  static std::map<void*, std::recursive_mutex*> m;
  std::lock_guard<std::mutex> lk(mu);
  auto it = m.find(stream);
  if (it == m.end()) it = m.emplace(stream, new std::recursive_mutex()).first;
  return *it->second;
}

mor_status solve_impl(const std::vector<mor_plan*>& plans, const std::vector<int>& plan_of, const double* ebar,
                      int64_t B, const mor_phase* phase, double tol, const mor_solve_opts* opts, mor_outputs* out,
                      float* jstate, int eff_stride, std::vector<RveState>* st_out,
                      unsigned char* arena = nullptr, size_t arena_cap = 0) {
  std::lock_guard<std::recursive_mutex> lk(stream_mutex(opts ? opts->stream : nullptr));
  SolveCtx cx;
  if (arena) {
    cx.noalloc = true;
    cx.arena = arena;
    cx.arena_cap = arena_cap;
  }
  mor_status s = setup(cx, plans, plan_of, ebar, B, phase, tol, opts, jstate);
  if (s != MOR_OK) {
    (void)hipStreamSynchronize(cx.st);
    return s;
  }
  cx.want_eps = out && out->strain;
  cx.want_sig = out && out->stress;
  s = run(cx, opts ? (const cpx<float>*)opts->warm_start : nullptr, opts, out ? out->strain : nullptr,
          out ? out->stress : nullptr);
  if (s != MOR_OK) {
    (void)hipStreamSynchronize(cx.st);
    return s;
  }
  return collect(cx, out, eff_stride, st_out);
}

}  // namespace

extern "C" mor_status mor_solve(mor_plan_t plan, const double* macro_strain, int64_t B, const mor_phase phase[2],
                                double tol, const mor_solve_opts* opts, mor_outputs* out) {
  if (!plan) {
    mor_set_error("mor_solve: NULL plan");
    return MOR_E_INVALID_ARG;
  }
  const int C = plan->ndim == 2 ? 3 : 6;
  mor_status s = check_common(macro_strain, B, C, phase, tol, opts, plan->ndim);
  if (s != MOR_OK) return s;
  std::vector<mor_plan*> plans = {plan};
  std::vector<int> plan_of(B, 0);
  return solve_impl(plans, plan_of, macro_strain, B, phase, tol, opts, out, nullptr, plan->ndim == 2 ? 4 : 6,
                    nullptr);
}

// ------------------------------------------------------------------ no-allocation solve
// The device scratch array of mor_solve_noalloc.  In host code its name is
// only a stand-in for the symbol: the device address is looked up once per
// device with hipGetSymbolAddress (each GPU holds its own copy) and only
// that address is passed to kernels and copies.
static __device__ __align__(256) unsigned char scratch[MOR_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_ptr;  // device -> address of its scratch array

mor_status scratch_address(unsigned char** out) {
  int dev = 0;
  MOR_HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return MOR_OK;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    mor_set_error(std::string("mor_solve_noalloc: hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    return MOR_E_DEVICE;
  }
  g_scratch_ptr[dev] = (unsigned char*)ptr;
  *out = (unsigned char*)ptr;
  return MOR_OK;
}
}  // namespace

extern "C" mor_status mor_solve_noalloc(mor_plan_t plan, const double* macro_strain, int64_t B,
                                        const mor_phase phase[2], double tol, const mor_solve_opts* opts,
                                        mor_outputs* out) {
  if (!plan) {
    mor_set_error("mor_solve_noalloc: NULL plan");
    return MOR_E_INVALID_ARG;
  }
  const int C = plan->ndim == 2 ? 3 : 6;
  mor_status s = check_common(macro_strain, B, C, phase, tol, opts, plan->ndim);
  if (s != MOR_OK) return s;
  if (opts && opts->use_graph) {
    mor_set_error("mor_solve_noalloc: use_graph records a graph per call; capture the call instead");
    return MOR_E_UNSUPPORTED;
  }
  unsigned char* base = nullptr;
  if ((s = scratch_address(&base)) != MOR_OK) return s;
  std::vector<mor_plan*> plans = {plan};
  std::vector<int> plan_of(B, 0);
  return solve_impl(plans, plan_of, macro_strain, B, phase, tol, opts, out, nullptr, plan->ndim == 2 ? 4 : 6,
                    nullptr, base, MOR_NOALLOC_SCRATCH_BYTES);
}

extern "C" mor_status mor_solve_multi(const mor_plan_t* plans, int64_t nplans, const int64_t* plan_of_rve,
                                      const double* macro_strain_packed, int64_t B, const mor_phase phase[2],
                                      double tol, const mor_solve_opts* opts, mor_outputs* out) {
  if (!plans || nplans < 1 || !plan_of_rve) {
    mor_set_error("mor_solve_multi: NULL or empty plan list");
    return MOR_E_INVALID_ARG;
  }
  for (int64_t i = 0; i < nplans; ++i)
    if (!plans[i]) {
      mor_set_error("mor_solve_multi: NULL plan");
      return MOR_E_INVALID_ARG;
    }
  const int ndim = plans[0]->ndim;
  for (int64_t i = 0; i < nplans; ++i)
    if (plans[i]->ndim != ndim) {
      mor_set_error("mor_solve_multi: all plans must have the same ndim");
      return MOR_E_UNSUPPORTED;
    }
  std::vector<int> plan_of(B > 0 ? B : 0);
  for (int64_t b = 0; b < B; ++b) {
    if (plan_of_rve[b] < 0 || plan_of_rve[b] >= nplans) {
      mor_set_error("mor_solve_multi: plan_of_rve out of range");
      return MOR_E_INVALID_ARG;
    }
    plan_of[b] = (int)plan_of_rve[b];
  }
  const int C = ndim == 2 ? 3 : 6;
  mor_status s = check_common(macro_strain_packed, B, C, phase, tol, opts, ndim);
  if (s != MOR_OK) return s;
  std::vector<mor_plan*> pl(plans, plans + nplans);
  return solve_impl(pl, plan_of, macro_strain_packed, B, phase, tol, opts, out, nullptr, ndim == 2 ? 4 : 6, nullptr);
}

// ------------------------------------------------------------------ compatibility step
// Coefficient index of every stored linear frequency of a plan (-1 where the
// plan stores none): cleared, then marked.
__global__ void k_fill_i32(int* __restrict__ p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_mark_coef(const int64_t* __restrict__ coef_lin, int ncoef, int* __restrict__ table) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ncoef) table[coef_lin[e]] = e;
}
// Reduced coefficients [B][C][ncr] placed at the same frequencies of the
// full set's layout [B][C][ncf] (cleared first); blockIdx.y = (b, c).
__global__ void k_embed_coef(const cpx<float>* __restrict__ in, const int64_t* __restrict__ lin_r, int ncr,
                             const int* __restrict__ table, int ncf, cpx<float>* __restrict__ out) {
  const int64_t bc = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncr) return;
  const int f = table[lin_r[e]];
  if (f >= 0) out[bc * ncf + f] = in[bc * ncr + e];
}
__global__ void k_zero_c64(cpx<float>* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = {0.f, 0.f};
}

extern "C" mor_status mor_compat(mor_plan_t plan, mor_plan_t plan_full, const float* coeffs,
                                 const double* macro_strain, int64_t B, const mor_phase phase[2], const float* state,
                                 const mor_solve_opts* opts, mor_outputs* out) {
  if (!plan || !plan_full || !coeffs) {
    mor_set_error("mor_compat: NULL plan or coefficients");
    return MOR_E_INVALID_ARG;
  }
  if (plan->ndim != plan_full->ndim || plan->n[0] != plan_full->n[0] || plan->n[1] != plan_full->n[1] ||
      plan->n[2] != plan_full->n[2] || plan->count != plan_full->count) {
    mor_set_error("mor_compat: plan_full must be a plan of the same grid and microstructure");
    return MOR_E_INVALID_ARG;
  }
  if (plan_full->M_actual != plan_full->N) {
    mor_set_error("mor_compat: plan_full must hold every frequency (M = N)");
    return MOR_E_INVALID_ARG;
  }
  const int C = plan->ndim == 2 ? 3 : 6;
  const int NST = plan->ndim == 2 ? 5 : 7;
  mor_status s = check_common(macro_strain, B, C, phase, 1.0, opts, plan->ndim);
  if (s != MOR_OK) return s;
  hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
  std::lock_guard<std::recursive_mutex> lk(stream_mutex(st));
  Workspace& ws = *workspace_for(st);
  const int64_t N = plan->N;
  const int ncr = plan->dev.ncoef, ncf = plan_full->dev.ncoef;
  int* table = nullptr;
  cpx<float>* warm = nullptr;
  if ((s = ws.get("compat_table", (size_t)N, &table)) != MOR_OK) return s;
  if ((s = ws.get("compat_warm", (size_t)B * C * ncf, &warm)) != MOR_OK) return s;
  k_fill_i32<<<(unsigned)std::min<int64_t>(4096, (N + 255) / 256), 256, 0, st>>>(table, N, -1);
  MOR_LAUNCH_CHECK("compat table");
  k_mark_coef<<<(ncf + 255) / 256, 256, 0, st>>>(plan_full->d_coef_lin, ncf, table);
  MOR_LAUNCH_CHECK("compat table");
  k_zero_c64<<<4096, 256, 0, st>>>(warm, B * C * (int64_t)ncf);
  MOR_LAUNCH_CHECK("compat clear");
  if (ncr > 0) {
    k_embed_coef<<<dim3((ncr + 255) / 256, (unsigned)(B * C)), 256, 0, st>>>((const cpx<float>*)coeffs,
                                                                              plan->d_coef_lin, ncr, table, ncf, warm);
    MOR_LAUNCH_CHECK("compat embed");
  }
  const bool j2 = phase[0].plastic || phase[1].plastic;
  float* jst = nullptr;
  if (j2) {
    // the committed state is used, not updated: the pass works on a copy
    if ((s = ws.get("compat_state", (size_t)B * NST * N, &jst)) != MOR_OK) return s;
    if (state)
      MOR_HIP_TRY(hipMemcpyAsync(jst, state, (size_t)B * NST * N * sizeof(float), hipMemcpyDeviceToDevice, st));
    else
      MOR_HIP_TRY(hipMemsetAsync(jst, 0, (size_t)B * NST * N * sizeof(float), st));
  }
  mor_solve_opts o{};
  if (opts) o = *opts;
  o.warm_start = (const float*)warm;
  o.max_iter = 1;
  o.check_every = 1;
  o.use_graph = 0;
  std::vector<mor_plan*> plans = {plan_full};
  std::vector<int> plan_of(B, 0);
  // one Green-operator pass: the stop test can only report "not converged"
  // (or a zero change), both are the intended single pass
  s = solve_impl(plans, plan_of, macro_strain, B, phase, std::numeric_limits<double>::min(), &o, out, jst,
                 plan->ndim == 2 ? 4 : 6, nullptr);
  if (s == MOR_E_NOT_CONVERGED) s = MOR_OK;
  return s;
}

namespace {
// Load paths of B RVEs in one set of launches per iteration (Secs. 2, 5.2):
// the context is prepared once; each step resets the per-RVE states and the
// macro strains on the device, starts from the previous step's coefficients
// (their zero-frequency entry becomes N times the new macro strain, i.e. the
// previous strain plus the macro increment), iterates every RVE to tolerance
// with the committed J2 state fixed, and commits the state in the final
// evaluation.  Effective stresses and states of every step are copied aside
// on the device and fetched once at the end.
//   macro: host [B][steps][C]; eff_out host [B][steps][eff_stride];
//   its/res host [B][steps].
mor_status path_impl(const std::vector<mor_plan*>& plans, const std::vector<int>& plan_of, const double* macro,
                     int64_t B, int steps, const mor_phase* phase, double tol, const mor_solve_opts* opts,
                     float* state, mor_outputs* out, int eff_stride) {
  std::lock_guard<std::recursive_mutex> lk(stream_mutex(opts ? opts->stream : nullptr));
  SolveCtx cx;
  const int C = plans[0]->ndim == 2 ? 3 : 6;
  std::vector<double> eb((size_t)B * C);
  auto step_ebar = [&](int n) {
    for (int64_t b = 0; b < B; ++b)
      for (int c = 0; c < C; ++c) eb[b * C + c] = macro[((size_t)b * steps + n) * C + c];
  };
  step_ebar(0);
  mor_status s = setup(cx, plans, plan_of, eb.data(), B, phase, tol, opts, state);
  if (s != MOR_OK) {
    (void)hipStreamSynchronize(cx.st);
    return s;
  }
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 10000;
  double* d_eff_hist = nullptr;
  RveState* d_st_hist = nullptr;
  if ((s = cx_get(cx, "eff_hist", (size_t)steps * B * cx.S, &d_eff_hist)) != MOR_OK) return s;
  if ((s = cx_get(cx, "st_hist", (size_t)steps * B, &d_st_hist)) != MOR_OK) return s;
  float* eps = out ? out->strain : nullptr;
  float* sig = out ? out->stress : nullptr;
  std::vector<std::vector<RveState>> hist((size_t)steps);
  for (int n = 0; n < steps; ++n) {
    const bool last = n == steps - 1;
    if (n > 0) {
      step_ebar(n);
      if ((s = upload(cx, cx.d_ebar, eb)) != MOR_OK) return s;
      if ((s = upload(cx, cx.d_st, fresh_states(cx, plans, plan_of, eb.data(), tol, max_iter))) != MOR_OK) return s;
      if ((s = upload(cx, cx.d_active, std::vector<unsigned int>(1, (unsigned int)B))) != MOR_OK) return s;
    }
    cx.want_eps = last && eps;
    cx.want_sig = last && sig;
    // step 0 starts from the caller's warm start (or cold), later steps from
    // the previous step's coefficients, read and rewritten in place
    const cpx<float>* warm = n == 0 ? (opts ? (const cpx<float>*)opts->warm_start : nullptr) : cx.d_coef;
    if ((s = run(cx, warm, opts, last ? eps : nullptr, last ? sig : nullptr)) != MOR_OK) {
      (void)hipStreamSynchronize(cx.st);
      return s;
    }
    MOR_HIP_TRY(hipMemcpyAsync(d_eff_hist + (size_t)n * B * cx.S, cx.d_eff, (size_t)B * cx.S * sizeof(double),
                               hipMemcpyDeviceToDevice, cx.st));
    MOR_HIP_TRY(hipMemcpyAsync(d_st_hist + (size_t)n * B, cx.d_st, (size_t)B * sizeof(RveState),
                               hipMemcpyDeviceToDevice, cx.st));
  }
  std::vector<double> effh((size_t)steps * B * cx.S);
  std::vector<RveState> sth((size_t)steps * B);
  MOR_HIP_TRY(hipMemcpyAsync(effh.data(), d_eff_hist, effh.size() * sizeof(double), hipMemcpyDeviceToHost, cx.st));
  MOR_HIP_TRY(hipMemcpyAsync(sth.data(), d_st_hist, sth.size() * sizeof(RveState), hipMemcpyDeviceToHost, cx.st));
  if (out && out->coeffs) {
    int64_t tot = 0;
    for (int64_t b = 0; b < B; ++b) tot += (int64_t)cx.C * cx.ncoef_h[b];
    MOR_HIP_TRY(hipMemcpyAsync(out->coeffs, cx.d_coef, tot * sizeof(cpx<float>), hipMemcpyDeviceToDevice, cx.st));
  }
  MOR_HIP_TRY(hipStreamSynchronize(cx.st));
  // profile: the recorded events of all steps, bytes from the summed iterations
  std::vector<RveState> tot_st(sth.begin(), sth.begin() + B);
  for (int n = 1; n < steps; ++n)
    for (int64_t b = 0; b < B; ++b) tot_st[b].iters += sth[(size_t)n * B + b].iters;
  account(cx, tot_st, steps);
  mor_status worst = MOR_OK;
  for (int64_t b = 0; b < B; ++b) {
    for (int n = 0; n < steps; ++n) {
      const RveState& r = sth[(size_t)n * B + b];
      const size_t k = (size_t)b * steps + n;
      if (out && out->iterations) out->iterations[k] = r.iters;
      if (out && out->residual) out->residual[k] = r.resid;
      if (out && out->eff_stress)
        for (int c = 0; c < cx.S; ++c) out->eff_stress[k * eff_stride + c] = effh[((size_t)n * B + b) * cx.S + c];
      if (r.status == MOR_E_NONFINITE) worst = MOR_E_NONFINITE;
      else if (r.status == MOR_E_NOT_CONVERGED && worst == MOR_OK) worst = MOR_E_NOT_CONVERGED;
    }
  }
  if (worst == MOR_E_NONFINITE) mor_set_error("non-finite residual in at least one load step");
  if (worst == MOR_E_NOT_CONVERGED) mor_set_error("max_iter reached before tol in at least one load step");
  return worst;
}
}  // namespace

extern "C" mor_status mor_solve_path(mor_plan_t plan, const double* macro_strain, int32_t steps,
                                     const mor_phase phase[2], double tol, const mor_solve_opts* opts, float* state,
                                     mor_outputs* out) {
  if (!plan || !state) {
    mor_set_error("mor_solve_path: NULL plan or state");
    return MOR_E_INVALID_ARG;
  }
  if (steps < 1) {
    mor_set_error("mor_solve_path: steps must be >= 1");
    return MOR_E_INVALID_ARG;
  }
  const int C = plan->ndim == 2 ? 3 : 6;
  const int S = plan->ndim == 2 ? 4 : 6;
  mor_status s = check_common(macro_strain, steps, C, phase, tol, opts, plan->ndim);
  if (s != MOR_OK) return s;
  std::vector<mor_plan*> plans = {plan};
  std::vector<int> plan_of(1, 0);
  return path_impl(plans, plan_of, macro_strain, 1, steps, phase, tol, opts, state, out, S);
}

extern "C" mor_status mor_solve_path_multi(const mor_plan_t* plans, int64_t nplans, const int64_t* plan_of_rve,
                                           const double* macro_strain, int64_t B, int32_t steps,
                                           const mor_phase phase[2], double tol, const mor_solve_opts* opts,
                                           float* state, mor_outputs* out) {
  if (!plans || nplans < 1 || !plan_of_rve || !state) {
    mor_set_error("mor_solve_path_multi: NULL or empty plan list, or NULL state");
    return MOR_E_INVALID_ARG;
  }
  if (steps < 1 || B < 1) {
    mor_set_error("mor_solve_path_multi: steps and B must be >= 1");
    return MOR_E_INVALID_ARG;
  }
  for (int64_t i = 0; i < nplans; ++i)
    if (!plans[i] || plans[i]->ndim != plans[0]->ndim) {
      mor_set_error("mor_solve_path_multi: NULL plan, or plans of different ndim");
      return MOR_E_INVALID_ARG;
    }
  std::vector<int> plan_of(B);
  for (int64_t b = 0; b < B; ++b) {
    if (plan_of_rve[b] < 0 || plan_of_rve[b] >= nplans) {
      mor_set_error("mor_solve_path_multi: plan_of_rve out of range");
      return MOR_E_INVALID_ARG;
    }
    plan_of[b] = (int)plan_of_rve[b];
  }
  const int C = plans[0]->ndim == 2 ? 3 : 6;
  mor_status s = check_common(macro_strain, B * (int64_t)steps, C, phase, tol, opts, plans[0]->ndim);
  if (s != MOR_OK) return s;
  std::vector<mor_plan*> pl(plans, plans + nplans);
  return path_impl(pl, plan_of, macro_strain, B, steps, phase, tol, opts, state, out, 6);
}

extern "C" mor_status mor_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return MOR_OK;
}

extern "C" mor_status mor_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& p : g_prof) p = ProfStat{};
  return MOR_OK;
}

extern "C" mor_status mor_profile_query(const char* kernel, double* total_ms, int64_t* launches, int64_t* items,
                                        double* bytes) {
  if (!kernel) {
    mor_set_error("mor_profile_query: NULL kernel name");
    return MOR_E_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int k = 0; k < PK_COUNT; ++k) {
    if (std::strcmp(kernel, kPkName[k]) == 0) {
      if (total_ms) *total_ms = g_prof[k].ms;
      if (launches) *launches = g_prof[k].launches;
      if (items) *items = g_prof[k].items;
      if (bytes) *bytes = g_prof[k].bytes;
      return MOR_OK;
    }
  }
  mor_set_error(std::string("mor_profile_query: unknown kernel ") + kernel);
  return MOR_E_INVALID_ARG;
}

// ------------------------------------------------------------------ kernel variants (ABI)
namespace {
int comps_of_ndim(int ndim) { return ndim == 2 ? 3 : ndim == 3 ? 6 : 0; }

// Variant table of (kernel, C, length): key size = half row length (row) or
// n0 (column).
int tune_count(int kernel, int C, int length) {
  if (C == 0 || length < 2) return 0;
  if (kernel == MOR_KERNEL_ROW) return (length & 1) ? 0 : row_variants(C, length / 2);
  if (kernel == MOR_KERNEL_COL) return col_variants(C, length);
  return 0;
}
std::map<std::pair<int, int>, int>& tune_table(int kernel) { return kernel == MOR_KERNEL_ROW ? g_row_var : g_col_var; }
std::pair<int, int> tune_key(int kernel, int C, int length) {
  return {C, kernel == MOR_KERNEL_ROW ? length / 2 : length};
}

mor_status check_tune_args(int32_t kernel, int32_t ndim, int32_t length, int* C, int* nh, const char* who) {
  *C = comps_of_ndim(ndim);
  *nh = length;
  if (tune_count(kernel, *C, length) == 0) {
    mor_set_error(std::string(who) + ": no tunable kernel for this (kernel, ndim, length)");
    return MOR_E_INVALID_ARG;
  }
  return MOR_OK;
}
}  // namespace

extern "C" mor_status mor_tune_variants(int32_t kernel, int32_t ndim, int32_t length, int32_t* count) {
  int C, nh;
  if (!count) {
    mor_set_error("mor_tune_variants: NULL count");
    return MOR_E_INVALID_ARG;
  }
  mor_status s = check_tune_args(kernel, ndim, length, &C, &nh, "mor_tune_variants");
  if (s != MOR_OK) return s;
  *count = tune_count(kernel, C, length);
  return MOR_OK;
}

extern "C" mor_status mor_tune_get(int32_t kernel, int32_t ndim, int32_t length, int32_t* variant) {
  int C, nh;
  if (!variant) {
    mor_set_error("mor_tune_get: NULL variant");
    return MOR_E_INVALID_ARG;
  }
  mor_status s = check_tune_args(kernel, ndim, length, &C, &nh, "mor_tune_get");
  if (s != MOR_OK) return s;
  std::lock_guard<std::mutex> lk(g_var_mu);
  auto& t = tune_table(kernel);
  auto it = t.find(tune_key(kernel, C, length));
  *variant = it == t.end() ? 0 : it->second;
  return MOR_OK;
}

extern "C" mor_status mor_tune_set(int32_t kernel, int32_t ndim, int32_t length, int32_t variant) {
  int C, nh;
  mor_status s = check_tune_args(kernel, ndim, length, &C, &nh, "mor_tune_set");
  if (s != MOR_OK) return s;
  if (variant < 0 || variant >= tune_count(kernel, C, length)) {
    mor_set_error("mor_tune_set: variant out of range");
    return MOR_E_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(g_var_mu);
  tune_table(kernel)[tune_key(kernel, C, length)] = variant;
  return MOR_OK;
}

extern "C" mor_status mor_tune_subbatch(int64_t bytes, int64_t min_rves, int64_t* prev_bytes, int64_t* prev_min) {
  if (bytes < -1 || min_rves < -1 || min_rves == 0) {
    mor_set_error("mor_tune_subbatch: bytes must be >= 0 and min_rves >= 1 (or -1 to keep)");
    return MOR_E_INVALID_ARG;
  }
  const int64_t ob = bytes < 0 ? subbatch_limit().load() : subbatch_limit().exchange(bytes);
  const int64_t om = min_rves < 0 ? subbatch_min_rves().load() : subbatch_min_rves().exchange(min_rves);
  if (prev_bytes) *prev_bytes = ob;
  if (prev_min) *prev_min = om;
  return MOR_OK;
}

// Autotuner: for every distinct row length among the plans, time `reps`
// batched solves of the given workload with each variant (the other sizes
// keep their current choice) and keep the fastest.  The workload's results
// are discarded; the tuned choice applies to later solves in this process.
extern "C" mor_status mor_autotune(const mor_plan_t* plans, int64_t nplans, const int64_t* plan_of_rve,
                                   const double* macro_strain_packed, int64_t B, const mor_phase phase[2],
                                   double tol, int32_t reps, void* stream) {
  if (!plans || nplans < 1 || !plan_of_rve || B < 1 || reps < 1 || !macro_strain_packed) {
    mor_set_error("mor_autotune: invalid argument");
    return MOR_E_INVALID_ARG;
  }
  // (kernel, ndim, length): the row kernel of every last-axis length and the
  // column kernel of every axis-0 length present
  std::vector<std::tuple<int, int, int>> sizes;
  for (int64_t i = 0; i < nplans; ++i) {
    if (!plans[i]) {
      mor_set_error("mor_autotune: NULL plan");
      return MOR_E_INVALID_ARG;
    }
    const int nd = plans[i]->ndim;
    for (auto key : {std::make_tuple((int)MOR_KERNEL_ROW, nd, plans[i]->n[nd - 1]),
                     std::make_tuple((int)MOR_KERNEL_COL, nd, plans[i]->n[0])})
      if (std::find(sizes.begin(), sizes.end(), key) == sizes.end()) sizes.push_back(key);
  }
  mor_solve_opts o{};
  o.stream = stream;
  const int C0 = comps_of_ndim(plans[0]->ndim);
  std::vector<double> eff((size_t)B * (C0 == 3 ? 4 : 6));
  std::vector<int32_t> its(B);
  std::vector<double> res(B);
  mor_outputs out{};
  out.eff_stress = eff.data();
  out.iterations = its.data();
  out.residual = res.data();
  for (auto [kernel, nd, len] : sizes) {
    const int C = comps_of_ndim(nd);
    const int nv = tune_count(kernel, C, len);
    if (nv < 2) continue;
    const auto key = tune_key(kernel, C, len);
    int best = 0;
    {
      std::lock_guard<std::mutex> lk(g_var_mu);
      auto it = tune_table(kernel).find(key);
      if (it != tune_table(kernel).end()) best = it->second;
    }
    double best_t = 1e300;
    for (int v = 0; v < nv; ++v) {
      {
        std::lock_guard<std::mutex> lk(g_var_mu);
        tune_table(kernel)[key] = v;
      }
      mor_status s = mor_solve_multi(plans, nplans, plan_of_rve, macro_strain_packed, B, phase, tol, &o, &out);
      if (s != MOR_OK && s != MOR_E_NOT_CONVERGED) return s;
      double tmin = 1e300;
      for (int r = 0; r < reps; ++r) {
        const auto t0 = std::chrono::steady_clock::now();
        s = mor_solve_multi(plans, nplans, plan_of_rve, macro_strain_packed, B, phase, tol, &o, &out);
        const auto t1 = std::chrono::steady_clock::now();
        if (s != MOR_OK && s != MOR_E_NOT_CONVERGED) return s;
        tmin = std::min(tmin, std::chrono::duration<double>(t1 - t0).count());
      }
      if (tmin < best_t) {
        best_t = tmin;
        best = v;
      }
    }
    std::lock_guard<std::mutex> lk(g_var_mu);
    tune_table(kernel)[key] = best;
  }
  return MOR_OK;
}
