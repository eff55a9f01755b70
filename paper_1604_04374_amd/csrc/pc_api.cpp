// Plan runtime and C ABI (include/pc.h).
//
// The plan turns the operator description of eq. 1.4 (m windows, m impulse
// responses, sizes) into device-resident data laid out for the kernels:
//   * 1D, N <= 8192: dense windows and full complex spectra F^* h_k;
//   * 1D four-step:  windows compacted to their circular support (the
//     compact-support idea of the complexity lemma of section 3.5 (Lemma 3.2)), spectra
//     in class-major order, in the frame of each window's origin o_k:
//     Hd[k][f1][f2] = H_k[f] W_N^{f o_k}, f = f1 + R f2;
//   * 2D:            window factors (or dense windows) and half-spectra
//     rfft2(h_k), N1 x (N2/2 + 1), row-major.
// All spectra are computed on the device by the library's own FFT kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <type_traits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "../../include/pc.h"
#include "fft_engine.hpp"
#include "pc_internal.hpp"

namespace {

thread_local std::string g_last_error;

}  // namespace
namespace pc {
uint64_t tune_key(const pc_plan_desc& d);
uint64_t tune_batch_key(const std::vector<pc_plan_desc>& ds);
}  // namespace pc
namespace {

// Default budget of the kept windowed spectra of a plan with gradients.
constexpr int64_t PC_DEFAULT_KEEP_BUDGET = (int64_t)1 << 30;

pc_status fail(pc_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

pc_status fail_hip(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return (e == hipErrorOutOfMemory) ? PC_ERROR_OUT_OF_MEMORY : PC_ERROR_HIP;
}

std::mutex g_registry_mu;
std::set<const void*> g_registry;  // live plans

// Twiddle table of the workgroup FFT engine for length L (see fft_engine.hpp):
// for each pass (stride Ns, radix R), exp(-2 i pi q k / (Ns R)) for k < Ns,
// 1 <= q < R, in float64 then rounded once.
std::vector<float2> engine_twiddles(int L, int P = 0) {
  if (P == 0) P = pc::points_per_thread(L);
  const pc::Sched s = pc::make_sched(L, P);
  std::vector<float2> tw;
  tw.reserve(L);
  long Ns = 1;
  for (int i = 0; i < s.n; ++i) {
    const int R = s.r[i];
    for (long k = 0; k < Ns; ++k)
      for (int q = 1; q < R; ++q) {
        const double a = -2.0 * M_PI * (double)(q * k) / (double)(Ns * R);
        tw.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
      }
    Ns *= R;
  }
  tw.push_back(make_float2(0.f, 0.f));  // pad to L entries
  return tw;
}

// exp(-2 i pi j / N), j < N, exact phase reduction in integers.
std::vector<float2> unit_roots(int64_t N) {
  std::vector<float2> w(N);
  for (int64_t j = 0; j < N; ++j) {
    const double a = -2.0 * M_PI * (double)j / (double)N;
    w[j] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  return w;
}

// Inner length L and class count R (N = R L, R in {2, 4, 8, 16}) of a
// four-step plan whose longest window support is max_support: the shortest L
// whose windows fit in two chunks of L samples (the short-support kernels;
// shorter transforms have fewer LDS exchanges, and at L = 4096 two
// workgroups share a compute unit), else the longest L (long-support path).
// A tuning entry for the workload overrides the choice.
bool large_split(int64_t N, int64_t max_support, int& L, int& R, uint64_t key = 0) {
  auto fits = [&](int l) {
    for (int r : {2, 4, 8, 16})
      if ((int64_t)l * r == N) {
        L = l;
        R = r;
        return true;
      }
    return false;
  };
  if (key) {  // a measured choice for this workload
    const int l = pc::tune_get(key, PC_TUNE_FOURSTEP_L, (int)N, 0);
    if (l && fits(l)) return true;
  }
  for (int l : {4096, 6144, 8192})
    if (max_support <= 2 * (int64_t)l && fits(l)) return true;
  for (int l : {8192, 6144, 4096})
    if (fits(l)) return true;
  return false;
}

// HIP-event tracer used while a plan's tracing is on.
struct PlanTracer final : pc::Tracer {
  struct Rec {
    std::string name;
    hipEvent_t a, b;
  };
  struct Stat {
    std::string name;
    int64_t n = 0;
    double tot = 0, mn = 0, mx = 0;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::vector<Stat> stats;
  std::string cur;
  hipEvent_t cur_a = nullptr;
  hipError_t err = hipSuccess;

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess && err == hipSuccess) err = r;
    return e;
  }
  void begin(const char* kernel, hipStream_t s) override {
    cur = kernel;
    cur_a = get();
    if (cur_a) {
      hipError_t r = hipEventRecord(cur_a, s);
      if (r != hipSuccess && err == hipSuccess) err = r;
    }
  }
  void end(hipStream_t s) override {
    hipEvent_t b = get();
    if (!b || !cur_a) return;
    hipError_t r = hipEventRecord(b, s);
    if (r != hipSuccess && err == hipSuccess) err = r;
    pending.push_back({cur, cur_a, b});
    cur_a = nullptr;
  }
  hipError_t flush() {
    for (Rec& r : pending) {
      float ms = 0.f;
      hipError_t e = hipEventSynchronize(r.b);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
      if (e != hipSuccess && err == hipSuccess) err = e;
      Stat* st = nullptr;
      for (Stat& x : stats)
        if (x.name == r.name) st = &x;
      if (!st) {
        stats.push_back(Stat{r.name});
        st = &stats.back();
      }
      if (st->n == 0 || ms < st->mn) st->mn = ms;
      if (st->n == 0 || ms > st->mx) st->mx = ms;
      st->tot += ms;
      st->n += 1;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
    hipError_t e = err;
    err = hipSuccess;
    return e;
  }
  ~PlanTracer() override {
    for (Rec& r : pending) {
      (void)hipEventSynchronize(r.b);
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct pc_plan_s {
  int device = 0;
  pc_plan_desc d{};
  int path = 0;
  int64_t n_total = 0;
  pc::Small1D s1{};
  pc::Large1D l1{};
  pc::Plan2D p2{};
  int64_t spectra_bytes = 0, window_bytes = 0, workspace_bytes = 0;
  std::vector<void*> allocs;
  bool tracing = false;
  PlanTracer tracer;
  float2* grad_ws = nullptr;  // PC_PLAN_GRADIENTS workspace
  int64_t spec_count = 0;     // complex values of the natural-layout spectra
  // product-convolution plan (eq. 1.3): built on the flipped responses, runs
  // the convolution-product directions exchanged; its stored spectra are
  // conj(F^* h_k), converted at the spectra calls through conj_ws
  bool pconv = false;
  float2* conj_ws = nullptr;
  // sectioned 2D (path 3): one single-term sub-plan per section, run through
  // an internal batch (its captured launch sequences)
  pc::Sec2D sec{};
  std::vector<pc_plan_s*> sec_sub;
  pc_batch_s* sec_batch = nullptr;
  int batch_refs = 0;  // live batches holding the plan (guarded by g_registry_mu)
  uint64_t tune_key = 0;  // workload key of the tuning table
  // What the last forward left for pc_backward: saved_state 1, the row
  // transforms of the windowed input saved_u (batch saved_batch) are still
  // in the workspace; 2, the windowed spectra U_k are also in keep.  Any
  // call that reuses the workspace resets it to 0.
  const float* saved_u = nullptr;
  int64_t saved_batch = 0;
  int saved_state = 0;
  // Kept windowed spectra U_k (PC_PLAN_GRADIENTS plans): held while they fit
  // in `budget` bytes (pc_plan_set_budget)
  int64_t budget = 0;
  int64_t keep_bytes = 0;
  void* keep_alloc = nullptr;
  // sectioned plans: section geometry (plan order), spectra transposes
  // (natural <-> each sub-plan's internal layout), and with gradients the
  // gradient export and the backward column launches [want_gu][kept U_k]
  std::vector<int> sec_k;
  std::vector<std::array<int64_t, 10>> sec_geom;  // o1 p1 o2 p2 a1 q1 a2 q2 M1 M2
  pc::TransposeSet tr_spec{};
  std::vector<pc::LaunchSet> sec_bwd[2][2];
  pc_batch_s* sec_batch_keep = nullptr;  // the forward launches storing U_k into keep
  std::vector<pc::SecTerm> sec_terms;
  // sectioned plans: the sections in two halves, whose launch chains run on
  // the call's stream and on sec_aux (forked and joined with events), so that
  // each pass of one half overlaps the other half's passes
  pc_batch_s* sec_half[2] = {nullptr, nullptr};
  hipStream_t sec_aux = nullptr;
  hipEvent_t sec_fork = nullptr, sec_join = nullptr;
  pc::Tracer* tr() { return tracing ? &tracer : nullptr; }

  ~pc_plan_s();

  template <class T>
  pc_status alloc(T** out, size_t count, int64_t* account = nullptr) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      *out = nullptr;
      return fail_hip(e, "hipMalloc");
    }
    allocs.push_back(p);
    *out = reinterpret_cast<T*>(p);
    if (account) *account += (int64_t)(count * sizeof(T));
    return PC_SUCCESS;
  }

  template <class T>
  pc_status upload(T** out, const std::vector<T>& host, hipStream_t s, int64_t* account = nullptr) {
    pc_status st = alloc(out, host.size(), account);
    if (st != PC_SUCCESS) return st;
    if (host.empty()) return PC_SUCCESS;
    (void)s;
    hipError_t e = hipMemcpy(*out, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpy");
    return PC_SUCCESS;
  }
};

// Plan-time staging buffer (impulse responses before their transform),
// freed once the spectra kernels have finished.
struct DeviceTemp {
  void* p = nullptr;
  ~DeviceTemp() {
    if (p) (void)hipFree(p);
  }
  pc_status upload(const float* host, size_t count) {
    hipError_t e = hipMalloc(&p, std::max<size_t>(count * sizeof(float), 256));
    if (e != hipSuccess) {
      p = nullptr;
      return fail_hip(e, "hipMalloc");
    }
    e = hipMemcpy(p, host, count * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpy");
    return PC_SUCCESS;
  }
  const float* get() const { return static_cast<const float*>(p); }
};

namespace {

pc_status check_plan(pc_plan p) {
  if (!p) return fail(PC_ERROR_INVALID_PLAN, "plan handle is NULL");
  std::lock_guard<std::mutex> g(g_registry_mu);
  if (!g_registry.count(p)) return fail(PC_ERROR_INVALID_PLAN, "plan handle is not a live plan");
  return PC_SUCCESS;
}

struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
      if (hipSetDevice(dev) == hipSuccess) changed = true;
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

// Minimal circular interval [o, o + S) holding every nonzero of w (S = 0 if
// w is identically zero).
void circular_support(const float* w, int64_t N, int64_t& o, int64_t& S) {
  int64_t first = -1;
  for (int64_t i = 0; i < N; ++i)
    if (w[i] != 0.0f) {
      first = i;
      break;
    }
  if (first < 0) {
    o = 0;
    S = 0;
    return;
  }
  // longest run of zeros on the circle, scanning from a nonzero
  int64_t best_len = 0, best_end = first, run = 0;
  for (int64_t t = 1; t <= N; ++t) {
    const int64_t i = (first + t) % N;
    if (w[i] == 0.0f) {
      ++run;
    } else {
      if (run > best_len) {
        best_len = run;
        best_end = i;  // first nonzero after the run
      }
      run = 0;
    }
  }
  o = best_len > 0 ? best_end : 0;
  S = N - best_len;
}

pc_status build_small1d(pc_plan p, const float* windows, const float* h, hipStream_t s) {
  const int L = (int)p->d.n0;
  const int m = p->d.m;
  pc_status st;
  float* w = nullptr;
  st = p->upload(&w, std::vector<float>(windows, windows + (size_t)m * L), s, &p->window_bytes);
  if (st) return st;
  float2* tw = nullptr;
  st = p->upload(&tw, engine_twiddles(L), s);
  if (st) return st;
  DeviceTemp hd;
  if ((st = hd.upload(h, (size_t)m * L))) return st;
  float2* H = nullptr;
  st = p->alloc(&H, (size_t)m * L, &p->spectra_bytes);
  if (st) return st;
  hipError_t e = pc::launch_spec1d_full(L, hd.get(), H, m, tw, s);
  if (e != hipSuccess) return fail_hip(e, "spectra kernel");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e, "spectra kernel");
  p->s1 = pc::Small1D{L, m, w, H, tw};
  return PC_SUCCESS;
}

pc_status build_large1d(pc_plan p, int L, int R, const float* windows, const float* h, hipStream_t s) {
  const int64_t N = (int64_t)L * R;
  const int m = p->d.m;
  const int64_t pairs = (p->d.batch + 1) / 2;
  pc_status st;
  // compacted windows and adjoint work items (term, chunk of <= L samples)
  std::vector<int> off(m), len(m);
  std::vector<int64_t> base(m);
  std::vector<float> wc;
  std::vector<int> it_k, it_d0, it_oc, it_len;
  std::vector<int64_t> it_out;
  int64_t pstride = 0;
  int64_t max_support = 0;
  for (int k = 0; k < m; ++k) {
    int64_t o, S;
    circular_support(windows + (size_t)k * N, N, o, S);
    off[k] = (int)o;
    len[k] = (int)S;
    max_support = std::max(max_support, S);
  }
  // short supports: windows within one or two chunks of L samples
  const int chunks = max_support <= L ? 1 : max_support <= 2 * (int64_t)L ? 2 : 0;
  for (int k = 0; k < m; ++k) {
    const float* wk = windows + (size_t)k * N;
    const int64_t o = off[k], S = len[k];
    base[k] = (int64_t)wc.size();
    for (int64_t d = 0; d < S; ++d) wc.push_back(wk[(o + d) % N]);
    // short-support plans keep every window on chunks x L samples (zeros
    // beyond its support) so that the fold loads every slot unconditionally
    if (chunks > 0) wc.resize((size_t)base[k] + (size_t)chunks * L, 0.f);
    // adjoint items: the whole support (short), or chunks of L samples (long)
    const int64_t step = chunks > 0 ? std::max<int64_t>(S, 1) : L;
    for (int64_t c0 = 0; c0 < S; c0 += step) {
      it_k.push_back(k);
      it_d0.push_back((int)c0);
      it_oc.push_back((int)((o + c0) % N));
      const int64_t cl = std::min<int64_t>(step, S - c0);
      it_len.push_back((int)cl);
      it_out.push_back(pstride);
      pstride += cl;
    }
  }
  // items that intersect each tile of 256 samples
  const int64_t n_tiles = N / 256;
  std::vector<int> tile_off(n_tiles + 1, 0), tile_items;
  {
    std::vector<std::vector<int>> lists(n_tiles);
    for (size_t i = 0; i < it_k.size(); ++i) {
      const int64_t a = it_oc[i], l = it_len[i];
      const int64_t t0 = a / 256, t1 = (a + l - 1) / 256;  // may run past n_tiles: wraps
      for (int64_t tt = t0; tt <= t1; ++tt) lists[tt % n_tiles].push_back((int)i);
    }
    for (int64_t tt = 0; tt < n_tiles; ++tt) {
      auto& v = lists[tt];
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
      tile_off[tt] = (int)tile_items.size();
      tile_items.insert(tile_items.end(), v.begin(), v.end());
    }
    tile_off[n_tiles] = (int)tile_items.size();
  }
  // class modulation table twC[f1 * L + n2] = exp(-2 i pi f1 n2 / N)
  std::vector<float2> twC((size_t)N);
  for (int f1 = 0; f1 < R; ++f1)
    for (int n2 = 0; n2 < L; ++n2) {
      const int64_t j = ((int64_t)f1 * n2) % N;
      const double a = -2.0 * M_PI * (double)j / (double)N;
      twC[(size_t)f1 * L + n2] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
  pc::Large1D& q = p->l1;
  q.L = L;
  q.R = R;
  q.P = pc::points_per_thread(L);
  if (!pc::fourstep_variant_supported(L, R, q.P)) return fail(PC_ERROR_UNSUPPORTED, "four-step variant not built");
  q.m = m;
  q.chunks = chunks;
  float* dwc = nullptr;
  if ((st = p->upload(&dwc, wc, s, &p->window_bytes))) return st;
  int *doff = nullptr, *dlen = nullptr, *dik = nullptr, *did0 = nullptr, *dioc = nullptr, *dilen = nullptr;
  int *dtoff = nullptr, *dtit = nullptr;
  int64_t *dbase = nullptr, *diout = nullptr;
  if ((st = p->upload(&doff, off, s))) return st;
  if ((st = p->upload(&dlen, len, s))) return st;
  if ((st = p->upload(&dbase, base, s))) return st;
  if ((st = p->upload(&dik, it_k, s))) return st;
  if ((st = p->upload(&did0, it_d0, s))) return st;
  if ((st = p->upload(&dioc, it_oc, s))) return st;
  if ((st = p->upload(&dilen, it_len, s))) return st;
  if ((st = p->upload(&diout, it_out, s))) return st;
  if ((st = p->upload(&dtoff, tile_off, s))) return st;
  if ((st = p->upload(&dtit, tile_items, s))) return st;
  float2 *tw = nullptr, *twN = nullptr, *dtwC = nullptr;
  if ((st = p->upload(&tw, engine_twiddles(L, q.P), s))) return st;
  if ((st = p->upload(&twN, unit_roots(N), s))) return st;
  if ((st = p->upload(&dtwC, twC, s))) return st;
  // short supports: window times class modulation per chunk, in the block
  // layout
  q.cw = nullptr;
  if (chunks > 0) {
    const int T = L / q.P;
    std::vector<float2> cw((size_t)m * N * chunks);
    for (int k = 0; k < m; ++k)
      for (int f1 = 0; f1 < R; ++f1)
        for (int c = 0; c < chunks; ++c) {
          float2* dst = cw.data() + (((size_t)k * R + f1) * chunks + c) * L;
          for (int d = 0; d < L; ++d) {
            const int64_t dd = (int64_t)c * L + d;
            const double wv = wc[(size_t)base[k] + dd];
            const double a = -2.0 * M_PI * (double)(((int64_t)f1 * dd) % N) / (double)N;
            dst[pc::block_pos(d, T)] = make_float2((float)(wv * std::cos(a)), (float)(wv * std::sin(a)));
          }
        }
    float2* dcw = nullptr;
    if ((st = p->upload(&dcw, cw, s, &p->window_bytes))) return st;
    q.cw = dcw;
  }
  q.wc = dwc;
  q.w_off = doff;
  q.w_len = dlen;
  q.w_base = dbase;
  q.tw = tw;
  q.twN = twN;
  q.twC = dtwC;
  float* zeros = nullptr;
  if ((st = p->upload(&zeros, std::vector<float>((size_t)N, 0.f), s, &p->workspace_bytes))) return st;
  q.zeros = zeros;
  q.n_items = (int)it_k.size();
  q.item_k = dik;
  q.item_d0 = did0;
  q.item_oc = dioc;
  q.item_len = dilen;
  q.item_out = diout;
  q.p_stride = pstride;
  q.tile_off = dtoff;
  q.tile_items = dtit;
  float2* Hd = nullptr;
  if ((st = p->alloc(&Hd, (size_t)m * N, &p->spectra_bytes))) return st;
  q.Hd = Hd;
  if ((st = p->alloc(&q.Bws, (size_t)pairs * N, &p->workspace_bytes))) return st;
  if ((st = p->alloc(&q.Vws, (size_t)pairs * N, &p->workspace_bytes))) return st;
  if ((st = p->alloc(&q.Pws, (size_t)pairs * std::max<int64_t>(pstride, 1), &p->workspace_bytes))) return st;
  DeviceTemp hd;
  if ((st = hd.upload(h, (size_t)m * N))) return st;
  hipError_t e = pc::launch_fold_fft(q, hd.get(), m, Hd, false, s);
  if (e == hipSuccess) e = pc::launch_origin_phase1d(q, Hd, s);
  if (e != hipSuccess) return fail_hip(e, "spectra kernel");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e, "spectra kernel");
  return PC_SUCCESS;
}

// Whether a column launch can take the single-term kernel: every job one
// term in one group, and (adjoint) transforming its own input; a forward
// launch that keeps U_k takes its KEEP variant.
template <class J>
bool single_term_cols(int kind, const std::vector<J>& jobs) {
  if constexpr (std::is_same<J, pc::ColJob>::value) {
    if (kind != pc::KK_COLS_FWD && kind != pc::KK_COLS_ADJ) return false;
    for (const pc::ColJob& j : jobs) {
      if (j.m1 * j.m2 != 1 || j.ngroups != 1) return false;
      if (kind == pc::KK_COLS_ADJ && !j.fft_src) return false;
    }
    return !jobs.empty();
  }
  return false;
}

// Most planes a row-inverse job of the list sums (0 for other jobs).
template <class J>
int max_planes(const std::vector<J>& jobs) {
  int n = 0;
  if constexpr (std::is_same<J, pc::RowJob>::value)
    for (const pc::RowJob& j : jobs) n = std::max(n, j.nq);
  return n;
}

template <class J>
pc_status make_set(pc_plan p, pc::LaunchSet& ls, int kind, int L, const std::vector<J>& jobs,
                   const std::vector<pc::BlockRef>& bm, int64_t per_img, const float2* tw, hipStream_t s,
                   bool small_rows = false, bool multi_term = true) {
  J* dj = nullptr;
  pc::BlockRef* db = nullptr;
  pc_status st = p->upload(&dj, jobs, s);
  if (st) return st;
  if ((st = p->upload(&db, bm, s))) return st;
  const bool rows = kind == pc::KK_ROWS_FWD || kind == pc::KK_ROWS_INV;
  ls.kind = kind;
  ls.L = L;
  ls.threads = rows ? pc::row_threads(L, small_rows) : pc::col_threads(L);
  ls.small_rows = rows && small_rows;
  const uint64_t key = p->tune_key;
  ls.late = kind == pc::KK_COLS_FWD && pc::tune_get(key, PC_TUNE_COLS_FWD_LATE, L, pc::cols_fwd_late(L, multi_term));
  ls.prefetch = kind == pc::KK_COLS_ADJ && pc::tune_get(key, PC_TUNE_COLS_ADJ_PREFETCH, L, pc::cols_adj_prefetch(L));
  ls.pipe = kind == pc::KK_ROWS_INV && pc::tune_get(key, PC_TUNE_ROWS_INV_PIPE, L, pc::rows_inv_pipe(L, ls.small_rows));
  ls.one = single_term_cols(kind, jobs);
  ls.one_plane = kind == pc::KK_ROWS_INV && max_planes(jobs) == 1;
  ls.jobs = dj;
  ls.bmap = db;
  ls.blocks = (int64_t)bm.size();
  ls.blocks_per_img = per_img;
  ls.tw = tw;
  return PC_SUCCESS;
}

// box: a single-term plan whose window is the product of a row factor and a
// column factor, given as [a[N1] | b[N2]] (windows unused): the row passes
// form the window from the two factors instead of reading a dense plane.
pc_status build_2d(pc_plan p, const float* windows, const float* h, hipStream_t s, const float* box = nullptr) {
  const int N1 = (int)p->d.n0, N2 = (int)p->d.n1, H2 = N2 / 2 + 1;
  const int m = p->d.m;
  const int64_t cap = p->d.batch;
  const bool dense = p->d.w_format == PC_W_DENSE;
  pc::Plan2D& q = p->p2;
  q.N1 = N1;
  q.N2 = N2;
  q.H2 = H2;
  q.m = m;
  q.dense = dense || box;
  q.wmode = box ? 3 : dense ? 2 : 1;
  q.batch_cap = cap;
  q.m1 = q.dense ? 1 : p->d.m_rows;
  q.m2 = q.dense ? m : p->d.m_cols;
  pc_status st;
  const int64_t plane = (int64_t)N1 * H2;
  if (box) {
    float* w = nullptr;
    if ((st = p->upload(&w, std::vector<float>(box, box + (size_t)N1 + N2), s, &p->window_bytes))) return st;
    q.wcols = w;
    q.wrows = nullptr;
  } else if (dense) {
    float* w = nullptr;
    if ((st = p->upload(&w, std::vector<float>(windows, windows + (size_t)m * N1 * N2), s, &p->window_bytes)))
      return st;
    q.wcols = w;
    q.wrows = nullptr;
  } else {
    float *a = nullptr, *b = nullptr;
    const size_t na = (size_t)q.m1 * N1, nb = (size_t)q.m2 * N2;
    if ((st = p->upload(&a, std::vector<float>(windows, windows + na), s, &p->window_bytes))) return st;
    if ((st = p->upload(&b, std::vector<float>(windows + na, windows + na + nb), s, &p->window_bytes))) return st;
    q.wrows = a;
    q.wcols = b;
  }
  float2 *tw1 = nullptr, *tw2 = nullptr;
  if ((st = p->upload(&tw1, engine_twiddles(N1), s))) return st;
  if (N2 == N1) {
    tw2 = tw1;
  } else if ((st = p->upload(&tw2, engine_twiddles(N2), s))) {
    return st;
  }
  q.tw1 = tw1;
  q.tw2 = tw2;
  float2* Hs = nullptr;
  if ((st = p->alloc(&Hs, (size_t)m * plane, &p->spectra_bytes))) return st;
  q.Hs = Hs;
  const int nq = q.dense ? m : q.m2;
  if ((st = p->alloc(&q.RA, (size_t)(nq * cap * plane), &p->workspace_bytes))) return st;
  if ((st = p->alloc(&q.Tws, (size_t)(cap * plane), &p->workspace_bytes))) return st;
  q.col_groups = std::max(1, std::min(nq, pc::tune_get(p->tune_key, PC_TUNE_COL_GROUPS, N1,
                                                        pc::col_groups_for(H2, cap, nq))));
  q.Part = nullptr;
  if (q.col_groups > 1 && (st = p->alloc(&q.Part, (size_t)(q.col_groups * cap * plane), &p->workspace_bytes)))
    return st;

  // launch tables
  const int mode = q.wmode;
  const float scale = 1.0f / ((float)N1 * (float)N2);
  // launches too small to fill the chip with the default row tiles (one row
  // block per compute unit at least) take the small tiles; the forward row
  // pass launches its blocks once per column factor
  // (a tuning entry for the workload decides instead)
  const bool sr = (int64_t)(N1 / pc::row_block_rows(N2)) * cap < 256;
  const int rpi = N1 / pc::row_block_rows(N2, sr);                 // row blocks per image
  const bool sr_q = pc::tune_get(p->tune_key, PC_TUNE_ROWS_FWD_SMALL, N2,
                                 (int64_t)(N1 / pc::row_block_rows(N2)) * cap * nq < 256);
  const int rpi_q = N1 / pc::row_block_rows(N2, sr_q);
  const bool sr_f = pc::tune_get(p->tune_key, PC_TUNE_ROWS_FWD_SMALL, N2, sr);   // adjoint's row-forward
  const int rpi_f = N1 / pc::row_block_rows(N2, sr_f);
  const bool sr_i = pc::tune_get(p->tune_key, PC_TUNE_ROWS_INV_SMALL, N2, sr);   // row-inverse passes
  const int rpi_i = N1 / pc::row_block_rows(N2, sr_i);
  const int cpi = (H2 + pc::col_block_cols(N1) - 1) / pc::col_block_cols(N1);  // column blocks per image
  std::vector<pc::BlockRef> bm;
  {  // forward: rows of b_q . u -> RA
    pc::RowJob j{nullptr, nullptr, q.wcols, mode, N1, 0, 0.f, nullptr, q.RA, plane * cap};
    bm.clear();
    pc::append_row_blocks(bm, 0, cap, N1, N2, nq, sr_q);
    if ((st = make_set(p, q.fwd_rows, pc::KK_ROWS_FWD, N2, std::vector<pc::RowJob>{j}, bm, (int64_t)rpi_q * nq, tw2, s,
                       sr_q)))
      return st;
  }
  pc::ColJob cf{q.RA, q.Tws, q.Part, Hs, q.wrows, plane * cap, plane * cap, H2, q.m1, q.m2, q.dense ? 1 : 0,
                q.col_groups};
  bm.clear();
  pc::append_col_blocks(bm, 0, cap, H2, N1, q.col_groups);
  if ((st = make_set(p, q.fwd_cols, pc::KK_COLS_FWD, N1, std::vector<pc::ColJob>{cf}, bm,
                     (int64_t)cpi * q.col_groups, tw1, s, false, m > 1)))
    return st;
  bm.clear();
  pc::append_col_blocks(bm, 0, cap, H2, N1, 1);
  if ((st = make_set(p, q.fwd_sum, pc::KK_COLS_SUM, N1, std::vector<pc::ColJob>{cf}, bm, cpi, tw1, s))) return st;
  {  // forward: rows of T -> y
    pc::RowJob j{nullptr, nullptr, nullptr, 0, N1, 1, scale, q.Tws, nullptr, 0};
    bm.clear();
    pc::append_row_blocks(bm, 0, cap, N1, N2, 1, sr_i);
    if ((st = make_set(p, q.fwd_rows_out, pc::KK_ROWS_INV, N2, std::vector<pc::RowJob>{j}, bm, rpi_i, tw2, s, sr_i)))
      return st;
  }
  {  // adjoint: rows of v -> Tws
    pc::RowJob j{nullptr, nullptr, nullptr, 0, N1, 0, 0.f, nullptr, q.Tws, plane * cap};
    bm.clear();
    pc::append_row_blocks(bm, 0, cap, N1, N2, 1, sr_f);
    if ((st = make_set(p, q.adj_rows, pc::KK_ROWS_FWD, N2, std::vector<pc::RowJob>{j}, bm, rpi_f, tw2, s, sr_f)))
      return st;
  }
  // a single term needs one column transform of V per column: the adjoint
  // column pass does it itself
  q.adj_fused = m == 1;
  pc::ColJob ca{q.Tws, q.RA, nullptr, Hs, q.wrows, plane * cap, 0, H2, q.m1, q.m2, q.dense ? 1 : 0, 1};
  ca.fft_src = q.adj_fused ? 1 : 0;
  pc::ColJob cfft{nullptr, q.Tws, nullptr, nullptr, nullptr, 0, 0, H2, q.m1, q.m2, q.dense ? 1 : 0, 1};
  bm.clear();
  pc::append_col_blocks(bm, 0, cap, H2, N1, 1);
  if ((st = make_set(p, q.adj_fft, pc::KK_COLS_FFT, N1, std::vector<pc::ColJob>{cfft}, bm, cpi, tw1, s))) return st;
  bm.clear();
  pc::append_col_blocks(bm, 0, cap, H2, N1, nq);
  if ((st = make_set(p, q.adj_cols, pc::KK_COLS_ADJ, N1, std::vector<pc::ColJob>{ca}, bm, (int64_t)cpi * nq, tw1, s)))
    return st;
  {  // adjoint: sum_q b_q . rows of Q_q -> x
    pc::RowJob j{nullptr, nullptr, q.wcols, mode, N1, nq, scale, q.RA, nullptr, plane * cap};
    bm.clear();
    pc::append_row_blocks(bm, 0, cap, N1, N2, 1, sr_i);
    if ((st = make_set(p, q.adj_rows_out, pc::KK_ROWS_INV, N2, std::vector<pc::RowJob>{j}, bm, rpi_i, tw2, s, sr_i)))
      return st;
  }
  {  // spectra: rows of h_k -> Hs, then columns in place
    pc::RowJob j{nullptr, nullptr, nullptr, 0, N1, 0, 0.f, nullptr, Hs, plane * m};
    bm.clear();
    pc::append_row_blocks(bm, 0, m, N1, N2, 1, sr);
    if ((st = make_set(p, q.spec_rows, pc::KK_ROWS_FWD, N2, std::vector<pc::RowJob>{j}, bm, rpi, tw2, s, sr))) return st;
    pc::ColJob c{nullptr, Hs, nullptr, nullptr, nullptr, 0, 0, H2, q.m1, q.m2, q.dense ? 1 : 0, 1};
    bm.clear();
    pc::append_col_blocks(bm, 0, m, H2, N1, 1);
    if ((st = make_set(p, q.spec_cols, pc::KK_COLS_FFT, N1, std::vector<pc::ColJob>{c}, bm, cpi, tw1, s))) return st;
  }
  DeviceTemp hd;
  if ((st = hd.upload(h, (size_t)m * N1 * N2))) return st;
  hipError_t e = pc::launch_spec2d(q, hd.get(), s);
  if (e != hipSuccess) return fail_hip(e, "spectra kernels");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e, "spectra kernels");
  return PC_SUCCESS;
}

bool overlaps(const void* a, const void* b, size_t bytes) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bytes && y < x + bytes;
}

pc_status check_apply(pc_plan p, const float* in, float* out, int64_t batch) {
  pc_status st = check_plan(p);
  if (st) return st;
  if (batch < 0 || batch > p->d.batch)
    return fail(PC_ERROR_INVALID_VALUE, "batch " + std::to_string(batch) + " outside [0, " +
                                            std::to_string(p->d.batch) + "]");
  if (batch == 0) return PC_SUCCESS;
  if (!in || !out) return fail(PC_ERROR_INVALID_VALUE, "input or output pointer is NULL");
  if (overlaps(in, out, (size_t)batch * p->n_total * sizeof(float)))
    return fail(PC_ERROR_INVALID_VALUE, "input and output buffers overlap");
  return PC_SUCCESS;
}

}  // namespace

struct pc_batch_s {
  int device = 0;
  uint64_t tune_key = 0;  // workload key of the tuning table (sections: the sectioned plan's)
  std::vector<pc_plan> plans;
  std::vector<void*> allocs;
  std::vector<pc::LaunchSet> fwd_seq, adj_seq;
  bool has_fwd = false, has_adj = false, use_graph = true;
  bool persistent = false;  // one persistent launch per pass for the lengths it holds code for
  hipGraph_t gf = nullptr, ga = nullptr;
  hipGraphExec_t ef = nullptr, ea = nullptr;
  // Buffers of the calls: the jobs read each instance's input and output
  // pointers from a device table, [direction][instance][in, out], refreshed
  // from pinned host staging before a call whose pointers differ from the
  // previous call's in that direction.
  float** dtab = nullptr;
  float** htab = nullptr;  // pinned host staging, same layout
  std::vector<float*> last[2];
  hipEvent_t ev[2] = {nullptr, nullptr};  // the last upload of each direction
  ~pc_batch_s() {
    if (ef) (void)hipGraphExecDestroy(ef);
    if (ea) (void)hipGraphExecDestroy(ea);
    if (gf) (void)hipGraphDestroy(gf);
    if (ga) (void)hipGraphDestroy(ga);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (htab) (void)hipHostFree(htab);
    for (void* p : allocs) (void)hipFree(p);
  }
  template <class T>
  pc_status upload(T** out, const std::vector<T>& host) {
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, std::max<size_t>(host.size() * sizeof(T), 256));
    if (e != hipSuccess) return fail_hip(e, "hipMalloc");
    allocs.push_back(d);
    e = hipMemcpy(d, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpy");
    *out = static_cast<T*>(d);
    return PC_SUCCESS;
  }
};

pc_plan_s::~pc_plan_s() {
  delete sec_batch;
  delete sec_batch_keep;
  delete sec_half[0];
  delete sec_half[1];
  if (sec_fork) (void)hipEventDestroy(sec_fork);
  if (sec_join) (void)hipEventDestroy(sec_join);
  if (sec_aux) (void)hipStreamDestroy(sec_aux);
  if (keep_alloc) (void)hipFree(keep_alloc);
  for (pc_plan_s* q : sec_sub) delete q;
  for (void* p : allocs) (void)hipFree(p);
}

namespace {

std::set<const void*> g_batches;  // live batches (guarded by g_registry_mu)

// Launch lists of one batch call.  Each call (apply, apply_adjoint) runs a
// forward-type chain (windowed row FFTs, term-split column pass with the
// spectral sum, inverse rows) for the instances that need the
// convolution-product direction, and an adjoint-type chain (row FFTs, column
// FFTs, per-(column, factor) adjoint columns, windowed inverse rows) for the
// others; a product-convolution plan takes the opposite chain of a
// convolution-product one.
struct BatchLists {
  std::vector<pc::LaunchSet> f_rows_in, f_cols, f_rows_out, a_rows_in, a_fft, a_cols, a_rows_out;
  // persistent passes (pc::PersistKind): their work items and lengths, and
  // the launches made of them
  std::vector<pc::PItem> items[4][3];  // [pass][length group]
  std::vector<int> lens[4][3];
  std::vector<pc::LaunchSet> persist[4];
};

template <class J>
pc_status batch_set(pc_batch b, std::vector<pc::LaunchSet>& seq, int kind, int L, const std::vector<J>& jobs,
                    const std::vector<pc::BlockRef>& bm, const float2* tw, bool multi_term = true,
                    bool small_rows = false, BatchLists* pl = nullptr, int pkind = -1, int psub = 0) {
  if (jobs.empty()) return PC_SUCCESS;
  J* dj = nullptr;
  pc::BlockRef* db = nullptr;
  pc_status st = b->upload(&dj, jobs);
  if (st) return st;
  if (pl && pkind >= 0 && b->persistent && pc::persist_length(L)) {
    // a length of the persistent pass: its blocks become work items
    const int g = pc::persist_group(L);
    for (const pc::BlockRef& r : bm) pl->items[pkind][g].push_back(pc::PItem{dj, r, tw, L, psub});
    if (std::find(pl->lens[pkind][g].begin(), pl->lens[pkind][g].end(), L) == pl->lens[pkind][g].end())
      pl->lens[pkind][g].push_back(L);
    return PC_SUCCESS;
  }
  if ((st = b->upload(&db, bm))) return st;
  pc::LaunchSet ls;
  const bool rows = kind == pc::KK_ROWS_FWD || kind == pc::KK_ROWS_INV;
  ls.kind = kind;
  ls.L = L;
  ls.threads = rows ? pc::row_threads(L, small_rows) : pc::col_threads(L);
  ls.small_rows = rows && small_rows;
  const uint64_t key = b->tune_key;
  ls.late = kind == pc::KK_COLS_FWD && pc::tune_get(key, PC_TUNE_COLS_FWD_LATE, L, pc::cols_fwd_late(L, multi_term));
  ls.prefetch = kind == pc::KK_COLS_ADJ && pc::tune_get(key, PC_TUNE_COLS_ADJ_PREFETCH, L, pc::cols_adj_prefetch(L));
  ls.pipe = kind == pc::KK_ROWS_INV && pc::tune_get(key, PC_TUNE_ROWS_INV_PIPE, L, pc::rows_inv_pipe(L, ls.small_rows));
  ls.one = single_term_cols(kind, jobs);
  ls.one_plane = kind == pc::KK_ROWS_INV && max_planes(jobs) == 1;
  ls.jobs = dj;
  ls.bmap = db;
  ls.blocks = (int64_t)bm.size();
  ls.tw = tw;
  seq.push_back(ls);
  return PC_SUCCESS;
}

hipError_t launch_seq(const std::vector<pc::LaunchSet>& seq, hipStream_t s, pc::Tracer* tr,
                      const float* x_arg = nullptr, int64_t img_limit = INT64_MAX, float* y_arg = nullptr) {
  for (const pc::LaunchSet& ls : seq) {
    hipError_t e = pc::launch_set(ls, ls.blocks, x_arg, y_arg, s, tr, img_limit);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

pc_status run_seq(const std::vector<pc::LaunchSet>& seq, hipStream_t s) {
  hipError_t e = launch_seq(seq, s, nullptr);
  if (e != hipSuccess) return fail_hip(e, "batch launch");
  return PC_SUCCESS;
}

pc_status capture(const std::vector<pc::LaunchSet>& seq, hipStream_t cs, hipGraph_t* g, hipGraphExec_t* ex) {
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return fail_hip(e, "hipStreamBeginCapture");
  pc_status st = run_seq(seq, cs);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  if (st) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
  *g = graph;
  e = hipGraphInstantiate(ex, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return fail_hip(e, "hipGraphInstantiate");
  return PC_SUCCESS;
}


// Section evaluation: the row-forward jobs read the boxes of the call's
// input in place (origins per instance: window box for apply, output box for
// the adjoint).
struct GatherSpec {
  int N1, N2;
  const std::vector<pc::SecTerm>* terms;
  // the window boxes partition the image: the adjoint's row-inverse pass
  // writes each section's window box straight into the call's output
  bool direct_adj = false;
};

// Block order for the XCDs.  Workgroup p of a launch runs on XCD p mod 8
// (workgroups are dealt to the 8 XCDs round-robin, each with its own L2).
// Blocks whose band key (band[i], one per block) is equal read the same
// lines; they are placed at positions of one residue mod 8, so that those
// lines are fetched into one L2 instead of several.  Every launch of the
// list still covers every block once, in an order that only the scheduling
// sees.
void xcd_group_blocks(std::vector<pc::BlockRef>& bm, const std::vector<int64_t>& band) {
  constexpr size_t X = 8;
  const size_t n = bm.size();
  std::vector<std::vector<size_t>> q(X);
  for (size_t i = 0; i < n; ++i) q[(size_t)(band[i] % (int64_t)X)].push_back(i);
  std::vector<pc::BlockRef> out;
  out.reserve(n);
  std::vector<size_t> head(X, 0);
  for (size_t p = 0; p < n; ++p) {
    size_t x = p % X;
    // the XCD's own blocks, else the next XCD's that has blocks left
    for (size_t k = 0; k < X && head[x] >= q[x].size(); ++k) x = (x + 1) % X;
    out.push_back(bm[q[x][head[x]++]]);
  }
  bm.swap(out);
}

// Fixed pointers (in, fo, fa: the sections of a sectioned plan) or, with
// in == nullptr, the entries of the batch's device table b->dtab.
pc_status build_batch(pc_batch b, const float* const* in, float* const* fo, float* const* fa,
                      const GatherSpec* gather = nullptr, const std::vector<float2*>* keep = nullptr) {
  const bool table = in == nullptr;
  const size_t nb = b->plans.size();  // rows of the pointer table
  // The instances: a full-grid plan is one; a sectioned plan contributes one
  // single-term instance per section, which reads its input box in place and
  // stages its output for the plan's overlap-add (or, adjoint with window
  // boxes that partition the image, writes the output itself).
  struct BInst {
    pc_plan q;              // the plan whose Plan2D runs (a section's sub-plan)
    size_t slot;            // its entry of the pointer table, or of in / fo / fa
    bool pconv;             // directions exchanged
    const pc::SecTerm* st;  // section geometry, or null
    int gN1, gN2;           // the section's image
    bool direct_adj;
    float* sout;            // the section's staging block (table mode)
  };
  std::vector<BInst> inst;
  for (size_t i = 0; i < nb; ++i) {
    pc_plan p = b->plans[i];
    if (gather) {
      inst.push_back({p, i, p->pconv, &(*gather->terms)[i], gather->N1, gather->N2, gather->direct_adj, nullptr});
    } else if (p->path == 3) {
      for (size_t k = 0; k < p->sec_sub.size(); ++k)
        inst.push_back({p->sec_sub[k], i, p->pconv, &p->sec_terms[k], p->sec.N1, p->sec.N2, p->sec.direct_adj,
                        p->sec.Sout + p->sec_terms[k].off});
    } else {
      inst.push_back({p, i, p->pconv, nullptr, 0, 0, false, nullptr});
    }
  }
  // group instances by row length (N2) and by column length (N1)
  std::vector<int> n2s, n1s;
  for (const BInst& x : inst) {
    if (std::find(n2s.begin(), n2s.end(), x.q->p2.N2) == n2s.end()) n2s.push_back(x.q->p2.N2);
    if (std::find(n1s.begin(), n1s.end(), x.q->p2.N1) == n1s.end()) n1s.push_back(x.q->p2.N1);
  }
  BatchLists lists[2];  // [0]: pc_batch_apply, [1]: pc_batch_apply_adjoint
  // Blocks are listed instance by instance, the instances with the most
  // terms first: a block's work grows with its instance's terms, and the
  // chip takes blocks roughly in list order, so the short blocks fill the
  // last, partly occupied round instead of the long ones.
  std::vector<size_t> order(inst.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t x, size_t y) { return inst[x].q->p2.m > inst[y].q->p2.m; });
  auto fwd_type = [&](size_t i, int c) { return (c == 0) != inst[i].pconv; };
  // a section instance whose chain ends in the staging block
  auto staged = [&](size_t i, int c) { return inst[i].st && (fwd_type(i, c) || !inst[i].direct_adj); };
  // instance i, call c: whether it runs (fixed pointers: a null output skips it)
  auto has = [&](size_t i, int c) { return table || (c == 0 ? fo[inst[i].slot] : fa[inst[i].slot]) != nullptr; };
  // its fixed output buffer (null: the table's, or the launch's argument)
  auto out_of = [&](size_t i, int c) -> float* {
    if (!table) return c == 0 ? fo[inst[i].slot] : fa[inst[i].slot];
    return staged(i, c) ? inst[i].sout : nullptr;
  };
  // the device table entries of instance i, call c
  auto in_slot = [&](size_t i, int c) -> const float* const* {
    return table ? const_cast<const float* const*>(b->dtab + (c * nb + inst[i].slot) * 2) : nullptr;
  };
  auto out_slot = [&](size_t i, int c) -> float* const* {
    return table && !staged(i, c) ? b->dtab + (c * nb + inst[i].slot) * 2 + 1 : nullptr;
  };
  pc_status st;
  for (int c = 0; c < 2; ++c) {
    BatchLists& bl = lists[c];
    for (int L2 : n2s) {
      const bool sf = pc::tune_get(b->tune_key, PC_TUNE_ROWS_FWD_SMALL, L2, 0) != 0;  // row tiles
      const bool si = pc::tune_get(b->tune_key, PC_TUNE_ROWS_INV_SMALL, L2, 0) != 0;
      // the persistent row passes take G = 256 / T row pairs per block, when
      // that many rows divide every image of this row length
      int pbr = b->persistent && pc::persist_length(L2) ? pc::persist_block_rows(L2) : 0;
      for (const BInst& x : inst)
        if (pbr && x.q->p2.N2 == L2 && x.q->p2.N1 % pbr) pbr = 0;
      BatchLists* prow = pbr ? &bl : nullptr;
      std::vector<pc::RowJob> jf, jfo, ja, jao;
      std::vector<pc::BlockRef> bf, bfo, ba, bao;
      const float2* tw = nullptr;
      for (size_t i : order) {
        const pc::Plan2D& q = inst[i].q->p2;
        float* out = out_of(i, c);
        if (q.N2 != L2 || !has(i, c)) continue;
        const float* inp = table ? nullptr : in[i];
        tw = q.tw2;
        const int64_t cap = q.batch_cap, plane = (int64_t)q.N1 * q.H2;
        const int nq = q.dense ? q.m : q.m2, mode = q.wmode;
        const float scale = 1.0f / ((float)q.N1 * (float)q.N2);
        auto gathered = [&](pc::RowJob j) {
          j.xp = in_slot(i, c);
          if (inst[i].st) {
            const pc::SecTerm& t = *inst[i].st;
            const bool f = fwd_type(i, c);
            j.x = nullptr;
            j.gN1 = inst[i].gN1;
            j.gN2 = inst[i].gN2;
            j.g1 = f ? t.gf1 : t.ga1;
            j.g2 = f ? t.gf2 : t.ga2;
          }
          return j;
        };
        // sections: rows that matter (the window box leads the section in
        // both directions; the forward output box is p + q - 1 rows)
        const pc::SecTerm* st = inst[i].st;
        const int win_rows = st ? st->ea1 : 0, out_rows = st ? st->ef1 : 0;
        if (fwd_type(i, c)) {
          pc::append_row_blocks(bf, (int)jf.size(), cap, q.N1, L2, nq, sf, win_rows, pbr);
          jf.push_back(gathered(pc::RowJob{inp, nullptr, q.wcols, mode, q.N1, 0, 0.f, nullptr, q.RA, plane * cap}));
          if (st) {  // samples outside the window box are zero and not read
            jf.back().mrows = st->ea1;
            jf.back().mcols = st->ea2;
          }
          pc::append_row_blocks(bfo, (int)jfo.size(), cap, q.N1, L2, 1, si, out_rows, pbr);
          pc::RowJob jo{nullptr, out, nullptr, 0, q.N1, 1, scale, q.Tws, nullptr, 0};
          jo.yp = out_slot(i, c);
          if (st) jo.ocols = st->ef2;  // the overlap-add reads the output box's columns only
          jfo.push_back(jo);
        } else {
          // sections: the rows of the forward output box only (the rest are zero)
          pc::append_row_blocks(ba, (int)ja.size(), cap, q.N1, L2, 1, sf, out_rows, pbr);
          ja.push_back(gathered(pc::RowJob{inp, nullptr, nullptr, 0, q.N1, 0, 0.f, nullptr, q.Tws, plane * cap}));
          if (st) {  // only the output box of the forward section is read (the gradient needs the mask)
            ja.back().mrows = st->ef1;
            ja.back().mcols = st->ef2;
          }
          pc::append_row_blocks(bao, (int)jao.size(), cap, q.N1, L2, 1, si, win_rows, pbr);
          pc::RowJob jo{nullptr, out, q.wcols, mode, q.N1, nq, scale, q.RA, nullptr, plane * cap};
          jo.yp = out_slot(i, c);
          if (st && inst[i].direct_adj) {
            jo.y = nullptr;  // the table's or the launch's output argument: the call's output image
            jo.oN1 = inst[i].gN1;
            jo.oN2 = inst[i].gN2;
            jo.o1 = st->sa1;
            jo.o2 = st->sa2;
            jo.orows = st->ea1;
            jo.ocols = st->ea2;
          }
          jao.push_back(jo);
        }
      }
      if ((st = batch_set(b, bl.f_rows_in, pc::KK_ROWS_FWD, L2, jf, bf, tw, true, sf, prow, pc::PK_ROWS_FWD)))
        return st;
      if ((st = batch_set(b, bl.f_rows_out, pc::KK_ROWS_INV, L2, jfo, bfo, tw, true, si, prow, pc::PK_ROWS_INV)))
        return st;
      if (gather && !prow && !ba.empty()) {
        // the sections' output boxes overlap: the adjoint's row-forward
        // blocks over the same image rows (same band of the row-block
        // height from the box origin) share their lines
        const int br = pc::row_block_rows(L2, sf);
        std::vector<int64_t> band(ba.size());
        for (size_t k = 0; k < ba.size(); ++k) {
          const pc::RowJob& j = ja[(size_t)ba[k].job];
          const int64_t r = ((int64_t)j.g1 + (int64_t)ba[k].blk * br) % (j.gN1 > 0 ? j.gN1 : 1);
          band[k] = (int64_t)ba[k].img * 1000003 + r / br;
        }
        xcd_group_blocks(ba, band);
      }
      if ((st = batch_set(b, bl.a_rows_in, pc::KK_ROWS_FWD, L2, ja, ba, tw, true, sf, prow, pc::PK_ROWS_FWD)))
        return st;
      if ((st = batch_set(b, bl.a_rows_out, pc::KK_ROWS_INV, L2, jao, bao, tw, true, si, prow, pc::PK_ROWS_INV)))
        return st;
    }
    for (int L1 : n1s) {
      std::vector<pc::ColJob> jf, jt, ja;
      std::vector<pc::BlockRef> bf, bt, ba;
      const float2* tw = nullptr;
      bool f_multi = false;  // some forward-type instance loops over several terms
      for (size_t i : order) {
        const pc::Plan2D& q = inst[i].q->p2;
        if (q.N1 != L1 || !has(i, c)) continue;
        tw = q.tw1;
        const int64_t cap = q.batch_cap, plane = (int64_t)q.N1 * q.H2;
        const int nq = q.dense ? q.m : q.m2, dense = q.dense ? 1 : 0;
        const pc::SecTerm* st = inst[i].st;
        if (fwd_type(i, c)) {  // one term group: the many instances already fill the device
          pc::append_col_blocks(bf, (int)jf.size(), cap, q.H2, L1, 1);
          f_multi = f_multi || q.m > 1;
          jf.push_back(pc::ColJob{q.RA, q.Tws, nullptr, q.Hs, q.wrows, plane * cap, 0, q.H2, q.m1, q.m2, dense, 1});
          if (st) {
            jf.back().nvalid_in = st->ea1;  // the row pass transformed the window box rows only
            // the row-inverse pass reads whole row blocks of the output box rows
            const int br = pc::row_block_rows(q.N2, pc::tune_get(b->tune_key, PC_TUNE_ROWS_INV_SMALL, q.N2, 0) != 0);
            jf.back().nvalid_out = std::min(q.N1, (st->ef1 + br - 1) / br * br);
          }
          if (keep) {
            jf.back().keep = (*keep)[i];
            jf.back().keep_stride = plane * cap;
          }
        } else {
          if (!q.adj_fused) {
            pc::append_col_blocks(bt, (int)jt.size(), cap, q.H2, L1, 1);
            jt.push_back(pc::ColJob{nullptr, q.Tws, nullptr, nullptr, nullptr, 0, 0, q.H2, q.m1, q.m2, dense, 1});
          }
          pc::append_col_blocks(ba, (int)ja.size(), cap, q.H2, L1, nq);
          pc::ColJob j{q.Tws, q.RA, nullptr, q.Hs, q.wrows, plane * cap, 0, q.H2, q.m1, q.m2, dense, 1};
          j.fft_src = q.adj_fused ? 1 : 0;
          if (st) {  // the row-inverse pass reads whole row blocks of the window box rows
            const int br = pc::row_block_rows(q.N2, pc::tune_get(b->tune_key, PC_TUNE_ROWS_INV_SMALL, q.N2, 0) != 0);
            j.nvalid_out = std::min(q.N1, (st->ea1 + br - 1) / br * br);
            j.nvalid_in = st->ef1;  // the row pass transformed the output box rows only
          }
          ja.push_back(j);
        }
      }
      const bool nokeep = keep == nullptr;  // the persistent forward column pass keeps nothing
      if ((st = batch_set(b, bl.f_cols, pc::KK_COLS_FWD, L1, jf, bf, tw, f_multi, false, nokeep ? &bl : nullptr,
                          pc::PK_COLS_A, 0)))
        return st;
      if ((st = batch_set(b, bl.a_fft, pc::KK_COLS_FFT, L1, jt, bt, tw, true, false, &bl, pc::PK_COLS_A, 1))) return st;
      if ((st = batch_set(b, bl.a_cols, pc::KK_COLS_ADJ, L1, ja, ba, tw, true, false, &bl, pc::PK_COLS_ADJ))) return st;
    }
  }
  for (int c = 0; c < 2; ++c) {
    BatchLists& bl = lists[c];
    for (int k = 0; k < 4; ++k)
      for (int g = 2; g >= 0; --g) {  // the launches of longer transforms first
      std::vector<pc::PItem>& it = bl.items[k][g];
      if (it.empty()) continue;
      // longer transforms first (within a length, the instances with the
      // most terms first, as listed)
      std::stable_sort(it.begin(), it.end(), [](const pc::PItem& x, const pc::PItem& y) { return x.L > y.L; });
      pc::PItem* di = nullptr;
      if ((st = b->upload(&di, it))) return st;
      pc::LaunchSet ls;
      ls.persist = k;
      ls.pgroup = g;
      ls.items = di;
      ls.n_items = (int)it.size();
      ls.lds_bytes = pc::persist_lds_bytes(k, bl.lens[k][g]);
      ls.blocks = pc::persist_grid(k, g, ls.lds_bytes, ls.n_items);
      ls.threads = pc::PERSIST_THREADS;
      ls.kind = k == pc::PK_ROWS_FWD ? pc::KK_ROWS_FWD : k == pc::PK_ROWS_INV ? pc::KK_ROWS_INV : pc::KK_COLS_FWD;
      bl.persist[k].push_back(ls);
      }
    std::vector<pc::LaunchSet>& seq = c == 0 ? b->fwd_seq : b->adj_seq;
    for (auto* v : {&bl.persist[pc::PK_ROWS_FWD], &bl.f_rows_in, &bl.a_rows_in, &bl.persist[pc::PK_COLS_A], &bl.f_cols,
                    &bl.a_fft, &bl.persist[pc::PK_COLS_ADJ], &bl.a_cols, &bl.persist[pc::PK_ROWS_INV], &bl.f_rows_out,
                    &bl.a_rows_out})
      seq.insert(seq.end(), v->begin(), v->end());
    // the overlap-add of each sectioned plan of a user batch, into the
    // table's output entry (a sectioned plan's own calls add it themselves)
    if (table)
      for (size_t i = 0; i < nb; ++i) {
        pc_plan p = b->plans[i];
        if (p->path != 3) continue;
        const bool fwd = (c == 0) != p->pconv;
        if (!fwd && p->sec.direct_adj) continue;  // the row-inverse pass wrote the output
        pc::LaunchSet ls;
        ls.kind = pc::KK_SEC_SCATTER;
        ls.sec = &p->sec;
        ls.sec_adjoint = !fwd;
        ls.sec_out = b->dtab + (c * nb + i) * 2 + 1;
        ls.blocks = p->sec.cap;  // images
        seq.push_back(ls);
      }
  }
  return PC_SUCCESS;
}

// ---------------------------------------------------------------------------
// Sectioned 2D plans (the compact-support complexity lemma of section 3.5)
// ---------------------------------------------------------------------------

// One section: term k with window box (o, p) and response lag box (a, q) per
// axis (origins mod N), evaluated on M1 x M2 samples.
struct Section {
  int k;
  int64_t o1, p1, o2, p2, a1, q1, a2, q2;
  int64_t M1, M2;
};

// circular supports of the nonzero rows and columns of a dense N1 x N2 array
void box_2d(const float* a, int64_t N1, int64_t N2, int64_t& o1, int64_t& p1, int64_t& o2, int64_t& p2) {
  std::vector<float> r((size_t)N1, 0.f), c((size_t)N2, 0.f);
  for (int64_t i = 0; i < N1; ++i)
    for (int64_t j = 0; j < N2; ++j)
      if (a[i * N2 + j] != 0.0f) {
        r[(size_t)i] = 1.f;
        c[(size_t)j] = 1.f;
      }
  circular_support(r.data(), N1, o1, p1);
  circular_support(c.data(), N2, o2, p2);
}

// smallest supported transform length >= need that is shorter than N, else N
int64_t section_len(int64_t need, int64_t N) {
  int64_t best = N;
  for (int64_t L = 64; L <= 8192; L *= 2)
    for (int64_t c : {L, 3 * L / 2})
      if (c >= need && c < best && pc::fft_size_supported(c)) best = c;
  return best;
}

// The sections of a 2D plan, if sectioning is at least twice as cheap as the
// full grid (transform work: two section transforms per term against m + 1
// full-grid transforms).
bool plan_sections(const pc_plan_desc& d, const float* windows, const float* h, std::vector<Section>& out) {
  const int64_t N1 = d.n0, N2 = d.n1;
  const bool dense = d.w_format == PC_W_DENSE;
  out.clear();
  double c_sec = 0.0;
  for (int k = 0; k < d.m; ++k) {
    Section sc{};
    sc.k = k;
    if (dense) {
      box_2d(windows + (size_t)k * N1 * N2, N1, N2, sc.o1, sc.p1, sc.o2, sc.p2);
    } else {
      const float* a = windows + (size_t)(k / d.m_cols) * N1;
      const float* b = windows + (size_t)d.m_rows * N1 + (size_t)(k % d.m_cols) * N2;
      circular_support(a, N1, sc.o1, sc.p1);
      circular_support(b, N2, sc.o2, sc.p2);
    }
    box_2d(h + (size_t)k * N1 * N2, N1, N2, sc.a1, sc.q1, sc.a2, sc.q2);
    if (sc.p1 == 0 || sc.p2 == 0 || sc.q1 == 0 || sc.q2 == 0) continue;  // the term is zero
    sc.M1 = section_len(sc.p1 + sc.q1 - 1, N1);
    sc.M2 = section_len(sc.p2 + sc.q2 - 1, N2);
    const double n = (double)sc.M1 * (double)sc.M2;
    c_sec += 2.0 * n * std::log2(n) + 4.0 * n;
    out.push_back(sc);
  }
  const double nf = (double)N1 * (double)N2;
  const double c_full = (double)(d.m + 1) * nf * std::log2(nf);
  return !out.empty() && 2.0 * c_sec < c_full;
}

pc_status create_plan(const pc_plan_desc& d, const float* windows, const float* h, hipStream_t s, pc_plan_s** out,
                      const float* box = nullptr);

pc_status make_transpose_set(pc_plan p, pc::TransposeSet& ts, std::vector<pc::TransposeJob> jobs) {
  int64_t b0 = 0;
  for (pc::TransposeJob& j : jobs) {
    j.block0 = b0;
    b0 += pc::transpose_blocks(j.N1, j.H2);
  }
  pc::TransposeJob* dj = nullptr;
  pc_status st = p->upload(&dj, jobs, nullptr);
  if (st) return st;
  ts.jobs = dj;
  ts.njobs = (int)jobs.size();
  ts.blocks = b0;
  return PC_SUCCESS;
}

// The backward column launches of a sectioned plan with gradients (one
// single-term job per section, grouped by column length), for the adjoint
// and spectra gradient together or the gradient alone; with kept U_k
// (kept = true, the sections' keep planes consecutive in keep_alloc) or
// recomputing them from the row transforms left in the workspace.
pc_status build_sec_bwd(pc_plan p, const std::vector<pc::SecTerm>& terms, bool kept) {
  const int64_t cap = p->d.batch;
  std::vector<int> lens;
  for (pc_plan_s* sub : p->sec_sub)
    if (std::find(lens.begin(), lens.end(), sub->p2.N1) == lens.end()) lens.push_back(sub->p2.N1);
  for (int gu = 0; gu < 2; ++gu) {
    std::vector<pc::LaunchSet>& seq = p->sec_bwd[gu][kept ? 1 : 0];
    seq.clear();
    for (int L1 : lens) {
      std::vector<pc::ColJob> jobs;
      std::vector<pc::BlockRef> bm;
      const float2* tw = nullptr;
      int64_t koff = 0, goff_next = 0;
      for (size_t i = 0; i < p->sec_sub.size(); ++i) {
        const pc::Plan2D& q = p->sec_sub[i]->p2;
        const int64_t plane = (int64_t)q.N1 * q.H2;
        float2* kp = kept ? static_cast<float2*>(p->keep_alloc) + koff : nullptr;
        koff += cap * plane;
        const int64_t goff = goff_next;
        goff_next += plane;
        if (q.N1 != L1) continue;
        tw = q.tw1;
        pc::ColJob j{q.Tws, q.RA, nullptr, q.Hs, nullptr, plane * cap, 0, q.H2, 1, 1, 1, 1};
        const pc::SecTerm& t = terms[i];
        const int br = pc::row_block_rows(q.N2, pc::tune_get(p->tune_key, PC_TUNE_ROWS_INV_SMALL, q.N2, 0) != 0);
        j.nvalid_in = t.ea1;
        j.nvalid_out = std::min(q.N1, (t.ea1 + br - 1) / br * br);
        j.nv_src = t.ef1;
        j.keep = kp;
        j.grad = p->sec_sub[i]->grad_ws;
        // the gradient straight into the caller's buffer, each section's
        // spectrum in its natural layout, one after another
        j.gext_off = goff;
        j.ginv_n = 1.0f / ((float)q.N1 * (float)q.N2);
        j.want_gu = gu;
        j.nimg = cap;
        pc::append_col_blocks(bm, (int)jobs.size(), 1, q.H2, L1, 1);
        jobs.push_back(j);
      }
      if (jobs.empty()) continue;
      pc::LaunchSet ls;
      pc_status st = make_set(p, ls, pc::KK_COLS_BWD1, L1, jobs, bm, 0, tw, nullptr);
      if (st) return st;
      ls.blocks_per_img = 0;
      seq.push_back(ls);
    }
  }
  return PC_SUCCESS;
}

// Whether the sections' window boxes (the adjoint's output boxes) cover
// every pixel of the N1 x N2 torus exactly once: their areas add up to the
// image and no two of them meet.
bool boxes_partition(const std::vector<pc::SecTerm>& t, int64_t N1, int64_t N2) {
  int64_t area = 0;
  for (const pc::SecTerm& a : t) area += (int64_t)a.ea1 * a.ea2;
  if (area != N1 * N2) return false;
  // circular intervals [s, s + e) and [s', s' + e') meet iff one starts
  // inside the other
  auto meet = [](int64_t s1, int64_t e1, int64_t s2, int64_t e2, int64_t n) {
    const int64_t d12 = ((s2 - s1) % n + n) % n, d21 = ((s1 - s2) % n + n) % n;
    return d12 < e1 || d21 < e2;
  };
  for (size_t i = 0; i < t.size(); ++i)
    for (size_t j = i + 1; j < t.size(); ++j)
      if (meet(t[i].sa1, t[i].ea1, t[j].sa1, t[j].ea1, N1) && meet(t[i].sa2, t[i].ea2, t[j].sa2, t[j].ea2, N2))
        return false;
  return true;
}

pc_status build_sec2d(pc_plan p, const float* windows, const float* h, const std::vector<Section>& secs,
                      hipStream_t s) {
  const pc_plan_desc& d = p->d;
  const int64_t N1 = d.n0, N2 = d.n1, cap = d.batch;
  const bool dense = d.w_format == PC_W_DENSE;
  pc::Sec2D& q = p->sec;
  q.N1 = (int)N1;
  q.N2 = (int)N2;
  q.cap = cap;
  q.n_sec = (int)secs.size();
  std::vector<pc::SecTerm> terms;
  int64_t off = 0;
  pc_status st;
  for (const Section& sc : secs) {
    // the single-term operator of the section: window box and shifted response
    std::vector<float> wsub((size_t)(sc.M1 * sc.M2), 0.f), hsub((size_t)(sc.M1 * sc.M2), 0.f);
    for (int64_t i = 0; i < sc.p1; ++i)
      for (int64_t j = 0; j < sc.p2; ++j) {
        const int64_t r = (sc.o1 + i) % N1, c = (sc.o2 + j) % N2;
        float v;
        if (dense) {
          v = windows[((size_t)sc.k * N1 + r) * N2 + c];
        } else {
          v = windows[(size_t)(sc.k / d.m_cols) * N1 + r] *
              windows[(size_t)d.m_rows * N1 + (size_t)(sc.k % d.m_cols) * N2 + c];
        }
        wsub[(size_t)(i * sc.M2 + j)] = v;
      }
    for (int64_t i = 0; i < sc.q1; ++i)
      for (int64_t j = 0; j < sc.q2; ++j)
        hsub[(size_t)(i * sc.M2 + j)] = h[((size_t)sc.k * N1 + (sc.a1 + i) % N1) * N2 + (sc.a2 + j) % N2];
    // the window box as a row factor times a column factor when that
    // product reproduces every float32 sample exactly (always, for
    // separable windows), so the row passes need no dense window plane
    std::vector<float> box((size_t)(sc.M1 + sc.M2), 0.f);
    bool factored = true;
    if (!dense) {
      for (int64_t i = 0; i < sc.p1; ++i) box[(size_t)i] = windows[(size_t)(sc.k / d.m_cols) * N1 + (sc.o1 + i) % N1];
      for (int64_t j = 0; j < sc.p2; ++j)
        box[(size_t)(sc.M1 + j)] = windows[(size_t)d.m_rows * N1 + (size_t)(sc.k % d.m_cols) * N2 + (sc.o2 + j) % N2];
    } else {
      // pivot: the largest sample; a = its column, b = its row over the pivot
      int64_t pi = 0, pj = 0;
      for (int64_t i = 0; i < sc.p1; ++i)
        for (int64_t j = 0; j < sc.p2; ++j)
          if (std::fabs(wsub[(size_t)(i * sc.M2 + j)]) > std::fabs(wsub[(size_t)(pi * sc.M2 + pj)])) {
            pi = i;
            pj = j;
          }
      const float piv = wsub[(size_t)(pi * sc.M2 + pj)];
      for (int64_t i = 0; i < sc.p1; ++i) box[(size_t)i] = wsub[(size_t)(i * sc.M2 + pj)];
      for (int64_t j = 0; j < sc.p2; ++j) box[(size_t)(sc.M1 + j)] = wsub[(size_t)(pi * sc.M2 + j)] / piv;
    }
    for (int64_t i = 0; i < sc.p1 && factored; ++i)
      for (int64_t j = 0; j < sc.p2; ++j)
        if (box[(size_t)i] * box[(size_t)(sc.M1 + j)] != wsub[(size_t)(i * sc.M2 + j)]) {
          factored = false;
          break;
        }
    pc_plan_desc sd{};
    sd.ndim = 2;
    sd.m = 1;
    sd.n0 = sc.M1;
    sd.n1 = sc.M2;
    sd.batch = cap;
    sd.w_format = PC_W_DENSE;
    sd.flags = PC_PLAN_FULL_GRID | (d.flags & PC_PLAN_GRADIENTS);
    pc_plan_s* sub = nullptr;
    if ((st = create_plan(sd, wsub.data(), hsub.data(), s, &sub, factored ? box.data() : nullptr))) return st;
    p->sec_sub.push_back(sub);
    p->spectra_bytes += sub->spectra_bytes;
    p->window_bytes += sub->window_bytes;
    p->workspace_bytes += sub->workspace_bytes;
    p->sec_k.push_back(sc.k);
    p->sec_geom.push_back({sc.o1, sc.p1, sc.o2, sc.p2, sc.a1, sc.q1, sc.a2, sc.q2, sc.M1, sc.M2});
    pc::SecTerm t{};
    t.off = off;
    t.M1 = (int)sc.M1;
    t.M2 = (int)sc.M2;
    t.gf1 = (int)sc.o1;
    t.gf2 = (int)sc.o2;
    t.ga1 = (int)((sc.o1 + sc.a1) % N1);
    t.ga2 = (int)((sc.o2 + sc.a2) % N2);
    t.sf1 = t.ga1;
    t.sf2 = t.ga2;
    t.ef1 = (int)std::min(sc.p1 + sc.q1 - 1, sc.M1);
    t.ef2 = (int)std::min(sc.p2 + sc.q2 - 1, sc.M2);
    t.sa1 = t.gf1;
    t.sa2 = t.gf2;
    t.ea1 = (int)sc.p1;
    t.ea2 = (int)sc.p2;
    // the row-forward pass reads the boxes in place with one wrap per axis
    if (t.M1 > N1 || t.M2 > N2 || t.gf1 >= N1 || t.gf2 >= N2)
      return fail(PC_ERROR_UNSUPPORTED, "section larger than the image");
    terms.push_back(t);
    off += cap * sc.M1 * sc.M2;
  }
  if ((st = p->alloc(&q.Sout, (size_t)off, &p->workspace_bytes))) return st;
  pc::SecTerm* dterms = nullptr;
  if ((st = p->upload(&dterms, terms, s))) return st;
  q.terms = dterms;
  // output tiles met by each section's output box, forward and adjoint
  const int64_t tr = N1 / pc::SEC_TILE_R, tc = N2 / pc::SEC_TILE_C;
  q.tiles2 = (int)tc;
  for (int dir = 0; dir < 2; ++dir) {
    std::vector<std::vector<int>> lists((size_t)(tr * tc));
    for (size_t k = 0; k < terms.size(); ++k) {
      const pc::SecTerm& t = terms[k];
      const int s1 = dir ? t.sa1 : t.sf1, s2 = dir ? t.sa2 : t.sf2;
      const int e1 = dir ? t.ea1 : t.ef1, e2 = dir ? t.ea2 : t.ef2;
      std::vector<char> rows((size_t)tr, 0), cols((size_t)tc, 0);
      for (int64_t i = 0; i < e1; ++i) rows[(size_t)(((s1 + i) % N1) / pc::SEC_TILE_R)] = 1;
      for (int64_t j = 0; j < e2; ++j) cols[(size_t)(((s2 + j) % N2) / pc::SEC_TILE_C)] = 1;
      for (int64_t a = 0; a < tr; ++a)
        if (rows[(size_t)a])
          for (int64_t b = 0; b < tc; ++b)
            if (cols[(size_t)b]) lists[(size_t)(a * tc + b)].push_back((int)k);
    }
    std::vector<int> toff(lists.size() + 1, 0), items;
    for (size_t t = 0; t < lists.size(); ++t) {
      toff[t] = (int)items.size();
      items.insert(items.end(), lists[t].begin(), lists[t].end());
    }
    toff[lists.size()] = (int)items.size();
    int *doff = nullptr, *dit = nullptr;
    if ((st = p->upload(&doff, toff, s))) return st;
    if ((st = p->upload(&dit, items, s))) return st;
    (dir ? q.ta_off : q.tf_off) = doff;
    (dir ? q.ta_items : q.tf_items) = dit;
  }
  // the sections' transforms as one batch: launch lists and captured graphs
  pc_batch_s* b = new (std::nothrow) pc_batch_s();
  if (!b) return fail(PC_ERROR_OUT_OF_MEMORY, "host allocation failed");
  p->sec_batch = b;
  b->device = p->device;
  b->tune_key = p->tune_key;
  b->plans.assign(p->sec_sub.begin(), p->sec_sub.end());
  b->has_fwd = b->has_adj = true;
  std::vector<const float*> in(terms.size(), nullptr);
  std::vector<float*> outs;
  for (const pc::SecTerm& t : terms) outs.push_back(q.Sout + t.off);
  GatherSpec gs{(int)N1, (int)N2, &terms};
  gs.direct_adj = q.direct_adj = boxes_partition(terms, N1, N2);
  // the launches take the call's input pointer, so they are not captured
  b->use_graph = false;
  if ((st = build_batch(b, in.data(), outs.data(), outs.data(), &gs))) return st;
  if (terms.size() >= 2 && pc::tune_get(p->tune_key, PC_TUNE_SEC_STREAMS, 0, 0)) {
    // the two halves (alternate sections), for the calls' two launch chains
    for (int h = 0; h < 2; ++h) {
      pc_batch_s* hb = new (std::nothrow) pc_batch_s();
      if (!hb) return fail(PC_ERROR_OUT_OF_MEMORY, "host allocation failed");
      p->sec_half[h] = hb;
      hb->device = p->device;
      hb->tune_key = p->tune_key;
      hb->has_fwd = hb->has_adj = true;
      hb->use_graph = false;
      std::vector<pc::SecTerm> ht;
      std::vector<const float*> hin;
      std::vector<float*> hout;
      for (size_t i = (size_t)h; i < terms.size(); i += 2) {
        hb->plans.push_back(p->sec_sub[i]);
        ht.push_back(terms[i]);
        hin.push_back(nullptr);
        hout.push_back(q.Sout + terms[i].off);
      }
      GatherSpec hs{(int)N1, (int)N2, &ht};
      hs.direct_adj = q.direct_adj;
      if ((st = build_batch(hb, hin.data(), hout.data(), hout.data(), &hs))) return st;
    }
    hipError_t e = hipStreamCreateWithFlags(&p->sec_aux, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->sec_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->sec_join, hipEventDisableTiming);
    if (e != hipSuccess) return fail_hip(e, "section streams");
  }
  // spectra as parameters: the sections' spectra, one after another, each in
  // the natural layout of its M1 x M2 grid
  {
    // (the backward's column kernels write the spectra gradient in the same
    // layout themselves)
    std::vector<pc::TransposeJob> jobs;
    int64_t off_c = 0;
    for (pc_plan_s* sub : p->sec_sub) {
      const pc::Plan2D& q2 = sub->p2;
      jobs.push_back({const_cast<float2*>(q2.Hs), off_c, q2.N1, q2.H2, 0, 1.f, 0});
      off_c += (int64_t)q2.N1 * q2.H2;
    }
    p->spec_count = off_c;
    if ((st = make_transpose_set(p, p->tr_spec, jobs))) return st;
  }
  p->sec_terms = terms;
  if (d.flags & PC_PLAN_GRADIENTS) return build_sec_bwd(p, terms, false);
  return PC_SUCCESS;
}

// Bytes of the windowed spectra U_k a plan with gradients can keep: every
// term's spectrum for the plan's batch capacity (2D full grid: m x batch
// planes; sectioned: one plane per section and image).  0: the path keeps
// nothing (1D, product-convolution).
int64_t keep_size(pc_plan p) {
  if (!(p->d.flags & PC_PLAN_GRADIENTS) || p->pconv) return 0;
  if (p->path == 2) return (int64_t)p->d.m * p->d.batch * p->p2.N1 * p->p2.H2 * (int64_t)sizeof(float2);
  if (p->path == 3) {
    int64_t n = 0;
    for (pc_plan_s* sub : p->sec_sub) n += p->d.batch * sub->p2.N1 * (int64_t)sub->p2.H2;
    return n * (int64_t)sizeof(float2);
  }
  return 0;
}

// Hold the kept U_k when they fit in the budget, release them otherwise.
pc_status set_keep(pc_plan p, int64_t budget) {
  p->budget = budget;
  const int64_t need = keep_size(p);
  // the budget bounds what is kept; the tuning table may prefer recomputing
  // even within it (keeping writes U_k in every forward and reads it back)
  const bool want = need > 0 && need <= budget && pc::tune_get(p->tune_key, PC_TUNE_KEEP, 0, 1) != 0;
  if (p->saved_state > 1) p->saved_state = 1;
  if (want == (p->keep_alloc != nullptr)) return PC_SUCCESS;
  if (!want) {
    hipError_t e = hipDeviceSynchronize();  // kernels of earlier calls may still use it
    (void)hipFree(p->keep_alloc);
    p->keep_alloc = nullptr;
    p->keep_bytes = 0;
    p->p2.keep = nullptr;
    delete p->sec_batch_keep;
    p->sec_batch_keep = nullptr;
    if (e != hipSuccess) return fail_hip(e, "hipDeviceSynchronize");
    return PC_SUCCESS;
  }
  hipError_t e = hipMalloc(&p->keep_alloc, (size_t)need);
  if (e != hipSuccess) {
    p->keep_alloc = nullptr;
    return fail(PC_ERROR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(need) + " bytes for the kept spectra");
  }
  p->keep_bytes = need;
  float2* kp = static_cast<float2*>(p->keep_alloc);
  pc_status st = PC_SUCCESS;
  if (p->path == 2) {
    pc::Plan2D& q = p->p2;
    const int64_t plane = (int64_t)q.N1 * q.H2;
    pc::ColJob cf{q.RA, q.Tws, q.Part, q.Hs, q.wrows, plane * q.batch_cap, plane * q.batch_cap, q.H2, q.m1, q.m2,
                  q.dense ? 1 : 0, q.col_groups};
    cf.keep = kp;
    cf.keep_stride = plane * q.batch_cap;
    std::vector<pc::BlockRef> bm;
    pc::append_col_blocks(bm, 0, q.batch_cap, q.H2, q.N1, q.col_groups);
    const int cpi = (q.H2 + pc::col_block_cols(q.N1) - 1) / pc::col_block_cols(q.N1);
    st = make_set(p, q.fwd_cols_keep, pc::KK_COLS_FWD, q.N1, std::vector<pc::ColJob>{cf}, bm,
                  (int64_t)cpi * q.col_groups, q.tw1, nullptr, false, q.m > 1);
    q.fwd_cols_keep.keep = true;
    if (!st) q.keep = kp;
  } else {
    std::vector<float2*> keeps;
    int64_t off = 0;
    for (pc_plan_s* sub : p->sec_sub) {
      keeps.push_back(kp + off);
      off += p->d.batch * sub->p2.N1 * (int64_t)sub->p2.H2;
    }
    pc_batch_s* b = new (std::nothrow) pc_batch_s();
    if (!b) return fail(PC_ERROR_OUT_OF_MEMORY, "host allocation failed");
    p->sec_batch_keep = b;
    b->device = p->device;
    b->tune_key = p->tune_key;
    b->plans.assign(p->sec_sub.begin(), p->sec_sub.end());
    b->has_fwd = b->has_adj = true;
    b->use_graph = false;
    std::vector<const float*> in(p->sec_terms.size(), nullptr);
    std::vector<float*> outs;
    for (const pc::SecTerm& t : p->sec_terms) outs.push_back(p->sec.Sout + t.off);
    GatherSpec gs{p->sec.N1, p->sec.N2, &p->sec_terms};
    gs.direct_adj = p->sec.direct_adj;
    st = build_batch(b, in.data(), outs.data(), outs.data(), &gs, &keeps);
    for (pc::LaunchSet& ls : b->fwd_seq)
      if (ls.kind == pc::KK_COLS_FWD) ls.keep = true;  // its jobs carry the keep pointers
    if (!st) st = build_sec_bwd(p, p->sec_terms, true);
  }
  if (st) {
    (void)hipFree(p->keep_alloc);
    p->keep_alloc = nullptr;
    p->keep_bytes = 0;
    p->p2.keep = nullptr;
    delete p->sec_batch_keep;
    p->sec_batch_keep = nullptr;
  }
  return st;
}

// The launch sets of a sequence with the given kind.
std::vector<pc::LaunchSet> of_kind(const std::vector<pc::LaunchSet>& seq, int kind) {
  std::vector<pc::LaunchSet> out;
  for (const pc::LaunchSet& ls : seq)
    if (ls.kind == kind) out.push_back(ls);
  return out;
}

// Sectioned backward pass: gu = H_m^* gy (if gu) and the sections' spectra
// gradient (if gspec) from one transform of each section's box of gy.
// state: what the forward left (see pc_plan_s::saved_state).
hipError_t run_sec_backward(pc_plan p, const float* u, const float* gy, float* gu, float2* gspec, int64_t batch,
                            int state, hipStream_t s) {
  const pc_batch_s* b = p->sec_batch;
  hipError_t e = hipSuccess;
  if (gspec && state == 0) e = launch_seq(of_kind(b->fwd_seq, pc::KK_ROWS_FWD), s, p->tr(), u, batch);
  if (e == hipSuccess) e = launch_seq(of_kind(b->adj_seq, pc::KK_ROWS_FWD), s, p->tr(), gy, batch);
  const bool kept = state == 2 && p->keep_alloc;
  // (the column kernels write the spectra gradient, if wanted, into gspec)
  if (e == hipSuccess)
    e = launch_seq(p->sec_bwd[gu ? 1 : 0][kept ? 1 : 0], s, p->tr(), nullptr, batch, reinterpret_cast<float*>(gspec));
  if (e == hipSuccess && gu) {
    e = launch_seq(of_kind(b->adj_seq, pc::KK_ROWS_INV), s, p->tr(), nullptr, batch, gu);
    if (e == hipSuccess && !p->sec.direct_adj) e = pc::launch_sec_scatter(p->sec, gu, true, batch, s, p->tr());
  }
  return e;
}

hipError_t run_sections(pc_plan p, const float* in, float* out, int64_t batch, bool adjoint, hipStream_t s) {
  hipError_t e;
  if (p->sec_half[0]) {
    // the second half's chain on sec_aux, between a fork and a join event
    e = hipEventRecord(p->sec_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->sec_aux, p->sec_fork, 0);
    for (int h = 1; h >= 0 && e == hipSuccess; --h) {
      const pc_batch_s* b = p->sec_half[h];
      e = launch_seq(adjoint ? b->adj_seq : b->fwd_seq, h ? p->sec_aux : s, p->tr(), in, batch, out);
    }
    if (e == hipSuccess) e = hipEventRecord(p->sec_join, p->sec_aux);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p->sec_join, 0);
  } else {
    const pc_batch_s* b = p->sec_batch;
    // blocks of images >= batch return at once in every pass
    e = launch_seq(adjoint ? b->adj_seq : b->fwd_seq, s, p->tr(), in, batch, out);
  }
  if (e != hipSuccess) return e;
  if (adjoint && p->sec.direct_adj) return hipSuccess;  // the row pass wrote the output
  return pc::launch_sec_scatter(p->sec, out, adjoint, batch, s, p->tr());
}

// The convolution-product directions of a plan (eq. 1.4 and its adjoint).
hipError_t run_forward(pc_plan p, const float* u, float* y, int64_t batch, hipStream_t s) {
  if (p->path == 0) return pc::launch_fwd1d_small(p->s1, u, y, batch, s, p->tr());
  if (p->path == 1) return pc::launch_fwd1d_large(p->l1, u, y, batch, s, p->tr());
  if (p->path == 3) return run_sections(p, u, y, batch, false, s);
  return pc::launch_fwd2d(p->p2, u, y, batch, s, p->tr());
}

hipError_t run_adjoint(pc_plan p, const float* v, float* x, int64_t batch, hipStream_t s) {
  if (p->path == 0) return pc::launch_adj1d_small(p->s1, v, x, batch, s, p->tr());
  if (p->path == 1) return pc::launch_adj1d_large(p->l1, v, x, batch, s, p->tr());
  if (p->path == 3) return run_sections(p, v, x, batch, true, s);
  return pc::launch_adj2d(p->p2, v, x, batch, s, p->tr());
}

pc_status check_batch(pc_batch b) {
  std::lock_guard<std::mutex> g(g_registry_mu);
  if (!b || !g_batches.count(b)) return fail(PC_ERROR_INVALID_VALUE, "batch handle is not a live batch");
  return PC_SUCCESS;
}

pc_status create_plan(const pc_plan_desc& d, const float* windows, const float* h, hipStream_t s, pc_plan_s** out,
                      const float* box) {
  if (d.ndim != 1 && d.ndim != 2) return fail(PC_ERROR_INVALID_VALUE, "ndim must be 1 or 2");
  if (d.m < 1) return fail(PC_ERROR_INVALID_VALUE, "m must be >= 1");
  if (d.batch < 1) return fail(PC_ERROR_INVALID_VALUE, "batch must be >= 1");
  if (d.flags & ~(uint32_t)(PC_PLAN_GRADIENTS | PC_PLAN_PRODUCT_CONVOLUTION | PC_PLAN_FULL_GRID))
    return fail(PC_ERROR_INVALID_VALUE, "unknown flag bits");
  if (d.n0 < 1 || d.n1 < 1) return fail(PC_ERROR_INVALID_VALUE, "sizes must be positive");
  if (d.w_format != PC_W_DENSE && d.w_format != PC_W_SEPARABLE)
    return fail(PC_ERROR_INVALID_VALUE, "unknown window format");
  int path = 0, L = 0, R = 1;
  if (d.ndim == 1) {
    if (d.n1 != 1) return fail(PC_ERROR_INVALID_VALUE, "1D plans need n1 == 1");
    if (d.w_format != PC_W_DENSE) return fail(PC_ERROR_INVALID_VALUE, "1D plans take dense windows");
    if (pc::fft_size_supported(d.n0)) {
      path = 0;
    } else if (large_split(d.n0, d.n0, L, R)) {  // a four-step size: now read the supports
      int64_t max_support = 0;
      for (int64_t k = 0; k < d.m; ++k) {
        int64_t o = 0, S = 0;
        circular_support(windows + (size_t)k * d.n0, d.n0, o, S);
        max_support = std::max(max_support, S);
      }
      large_split(d.n0, max_support, L, R, pc::tune_key(d));
      path = 1;
    } else {
      return fail(PC_ERROR_UNSUPPORTED, "1D size " + std::to_string(d.n0) + " is not supported");
    }
  } else {
    if (!pc::fft_size_supported(d.n0) || !pc::fft_size_supported(d.n1))
      return fail(PC_ERROR_UNSUPPORTED,
                  "2D size " + std::to_string(d.n0) + "x" + std::to_string(d.n1) + " is not supported");
    if (d.w_format == PC_W_SEPARABLE &&
        (d.m_rows < 1 || d.m_cols < 1 || (int64_t)d.m_rows * d.m_cols != d.m))
      return fail(PC_ERROR_INVALID_VALUE, "separable windows need m == m_rows * m_cols");
    path = 2;
  }
  pc_plan_s* p = new (std::nothrow) pc_plan_s();
  if (!p) return fail(PC_ERROR_OUT_OF_MEMORY, "host allocation failed");
  p->d = d;
  p->path = path;
  p->n_total = d.n0 * d.n1;
  p->tune_key = pc::tune_key(d);
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return fail_hip(e, "hipGetDevice");
  }
  p->pconv = (d.flags & PC_PLAN_PRODUCT_CONVOLUTION) != 0;
  // G_m = (convolution-product operator of the flipped responses)^*
  std::vector<float> flipped;
  if (p->pconv) {
    const int64_t n0 = d.n0, n1 = d.n1;
    flipped.resize((size_t)d.m * n0 * n1);
    for (int64_t k = 0; k < d.m; ++k)
      for (int64_t i = 0; i < n0; ++i)
        for (int64_t j = 0; j < n1; ++j)
          flipped[(size_t)((k * n0 + i) * n1 + j)] = h[(size_t)((k * n0 + (n0 - i) % n0) * n1 + (n1 - j) % n1)];
    h = flipped.data();
  }
  std::vector<Section> secs;
  // sections: unless the full grid is asked for, or gradients of a
  // product-convolution plan (whose gradient needs both chains swapped)
  const bool grads = (d.flags & PC_PLAN_GRADIENTS) != 0;
  if (path == 2 && !(d.flags & PC_PLAN_FULL_GRID) && !(grads && p->pconv) && plan_sections(d, windows, h, secs))
    p->path = path = 3;
  pc_status st;
  if (path == 0)
    st = build_small1d(p, windows, h, s);
  else if (path == 1)
    st = build_large1d(p, L, R, windows, h, s);
  else if (path == 2)
    st = build_2d(p, windows, h, s, box);
  else
    st = build_sec2d(p, windows, h, secs, s);
  if (st == PC_SUCCESS && path != 3) {  // sectioned plans count their sections' spectra
    p->spec_count = (int64_t)d.m * (d.ndim == 1 ? d.n0 / 2 + 1 : d.n0 * (d.n1 / 2 + 1));
    if (p->pconv) st = p->alloc(&p->conj_ws, (size_t)p->spec_count, &p->workspace_bytes);
  }
  if (st == PC_SUCCESS && path != 3) {  // sections hold their gradient planes in their sub-plans
    if (d.flags & PC_PLAN_GRADIENTS) {
      // 1D: pair spectra (pairs x N) or the per-class accumulators (m x N); 2D: m planes
      const int64_t pairs = (d.batch + 1) / 2;
      const int64_t n = path == 0 ? pairs * d.n0 : path == 1 ? (int64_t)d.m * d.n0 : d.m * d.n0 * (d.n1 / 2 + 1);
      st = p->alloc(&p->grad_ws, (size_t)n, &p->workspace_bytes);
    }
  }
  if (st == PC_SUCCESS && grads) st = set_keep(p, PC_DEFAULT_KEEP_BUDGET);
  if (st != PC_SUCCESS) {
    (void)hipStreamSynchronize(s);
    delete p;
    return st;
  }
  *out = p;
  return PC_SUCCESS;
}

// Device scratch of the construction and wavelet calls, kept between calls:
// one grow-only buffer per device (allocating and freeing ~100 MB per call
// cost more than the solves).  A call holds its device's lock from commit()
// until it has waited for its stream, so calls on one device run one at a
// time and never share live scratch.
struct DeviceScratch {
  std::mutex mu;
  void* p = nullptr;
  size_t bytes = 0;
};
DeviceScratch& device_scratch(int device) {
  static DeviceScratch per_device[64];
  return per_device[device & 63];
}

// Temporary device buffers of one call: alloc() and upload() record the
// requests, commit() carves them out of the device scratch (256-byte
// aligned) and performs the uploads; the pointers are valid after commit().
struct CallTemps {
  struct Req {
    void** out;
    size_t bytes;
    const void* host;  // upload source, or null
  };
  std::vector<Req> reqs;
  DeviceScratch* sc = nullptr;
  hipStream_t stream = nullptr;
  ~CallTemps() {
    if (sc) {
      (void)hipStreamSynchronize(stream);  // nothing in flight uses the scratch
      sc->mu.unlock();
    }
  }
  template <class T>
  pc_status alloc(T** out, size_t count) {
    reqs.push_back(Req{reinterpret_cast<void**>(out), count * sizeof(T), nullptr});
    return PC_SUCCESS;
  }
  template <class T>
  pc_status upload(T** out, const T* host, size_t count) {
    reqs.push_back(Req{reinterpret_cast<void**>(out), count * sizeof(T), host});
    return PC_SUCCESS;
  }
  pc_status commit(hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(PC_ERROR_UNSUPPORTED, "device index above 63");
    size_t total = 0;
    for (const Req& r : reqs) total += (std::max<size_t>(r.bytes, 1) + 255) / 256 * 256;
    sc = &device_scratch(dev);
    sc->mu.lock();
    stream = s;
    if (total > sc->bytes) {  // the previous holder waited for its stream
      if (sc->p) (void)hipFree(sc->p);
      sc->p = nullptr;
      sc->bytes = 0;
      e = hipMalloc(&sc->p, total);
      if (e != hipSuccess) {
        sc->p = nullptr;
        return fail_hip(e, "hipMalloc");
      }
      sc->bytes = total;
    }
    char* base = static_cast<char*>(sc->p);
    for (const Req& r : reqs) {
      *r.out = base;
      if (r.host && r.bytes) {
        e = hipMemcpy(base, r.host, r.bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail_hip(e, "hipMemcpy");
      }
      base += (std::max<size_t>(r.bytes, 1) + 255) / 256 * 256;
    }
    return PC_SUCCESS;
  }
};

pc_status check_construct(int64_t n, int32_t m, int64_t rows, const void* a, const float* windows,
                                 const float* h, const int64_t* lags) {
  if (!a || !windows || !h || !lags) return fail(PC_ERROR_INVALID_VALUE, "null pointer");
  if (n < 16 || n % 16) return fail(PC_ERROR_INVALID_VALUE, "n must be a positive multiple of 16");
  if (m < 1 || m > pc::CONSTRUCT_MAX_M)
    return fail(PC_ERROR_INVALID_VALUE, "m must be in [1, " + std::to_string(pc::CONSTRUCT_MAX_M) + "]");
  if (rows < 1 || rows > n) return fail(PC_ERROR_INVALID_VALUE, "rows must be in [1, n]");
  std::vector<char> seen((size_t)n, 0);
  for (int64_t r = 0; r < rows; ++r) {
    if (lags[r] < 0 || lags[r] >= n || seen[(size_t)lags[r]])
      return fail(PC_ERROR_INVALID_VALUE, "lags must be distinct and in [0, n)");
    seen[(size_t)lags[r]] = 1;
  }
  return PC_SUCCESS;
}

pc_status finish_construct(hipStream_t s, const int* dfail, const char* what) {
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e, what);
  int bad = 0;
  e = hipMemcpy(&bad, dfail, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e, what);
  if (bad) return fail(PC_ERROR_INVALID_VALUE, std::string(what) + ": the windows' system is singular");
  return PC_SUCCESS;
}

pc_status make_filter(int32_t taps, const float* lowpass, pc::WaveletFilter& f) {
  if (!lowpass) return fail(PC_ERROR_INVALID_VALUE, "lowpass is NULL");
  if (taps < 2 || taps > pc::WAVELET_MAX_TAPS || taps % 2)
    return fail(PC_ERROR_INVALID_VALUE, "taps must be even, in [2, " + std::to_string(pc::WAVELET_MAX_TAPS) + "]");
  f.taps = taps;
  for (int k = 0; k < taps; ++k) {
    f.h[k] = lowpass[k];
    f.g[k] = (k % 2 ? -1.f : 1.f) * lowpass[taps - 1 - k];
  }
  return PC_SUCCESS;
}

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

}  // namespace

extern "C" {

pc_status pc_batch_create(pc_batch* out, int32_t count, const pc_plan* plans, uint32_t flags, void* stream) {
  if (!out) return fail(PC_ERROR_INVALID_VALUE, "out is NULL");
  *out = nullptr;
  if (count < 1 || !plans) return fail(PC_ERROR_INVALID_VALUE, "count < 1 or null plan array");
  if (flags & ~(uint32_t)(PC_BATCH_NO_GRAPH | PC_BATCH_PERSISTENT))
    return fail(PC_ERROR_INVALID_VALUE, "unknown flag bits");
  int device = -1;
  std::set<pc_plan> seen;
  for (int i = 0; i < count; ++i) {
    pc_status st = check_plan(plans[i]);
    if (st) return st;
    const pc_plan p = plans[i];
    if (!seen.insert(p).second)
      return fail(PC_ERROR_INVALID_VALUE, "plan of instance " + std::to_string(i) +
                                              " appears twice (instances share a plan's workspace)");
    if (p->path != 2 && p->path != 3) return fail(PC_ERROR_INVALID_VALUE, "batches take 2D plans");
    if (device < 0) device = p->device;
    if (p->device != device) return fail(PC_ERROR_INVALID_VALUE, "plans of a batch must share a device");
  }
  pc_batch_s* b = new (std::nothrow) pc_batch_s();
  if (!b) return fail(PC_ERROR_OUT_OF_MEMORY, "host allocation failed");
  b->device = device;
  b->plans.assign(plans, plans + count);
  b->has_fwd = b->has_adj = true;
  {
    std::vector<pc_plan_desc> ds;
    for (pc_plan q : b->plans) ds.push_back(q->d);
    b->tune_key = pc::tune_batch_key(ds);
  }
  b->persistent = (flags & PC_BATCH_PERSISTENT) || pc::tune_get(b->tune_key, PC_TUNE_BATCH_PERSISTENT, 0, 0) != 0;
  b->use_graph = !(flags & PC_BATCH_NO_GRAPH);
  DeviceGuard g(device);
  const size_t tab_bytes = (size_t)4 * count * sizeof(float*);
  pc_status st = PC_SUCCESS;
  {
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, tab_bytes);
    if (e != hipSuccess) {
      st = fail_hip(e, "hipMalloc");
    } else {
      b->allocs.push_back(d);
      b->dtab = static_cast<float**>(d);
      void* h = nullptr;
      e = hipHostMalloc(&h, tab_bytes, hipHostMallocDefault);
      if (e != hipSuccess) st = fail_hip(e, "hipHostMalloc");
      b->htab = static_cast<float**>(h);
      for (int c = 0; c < 2 && !st; ++c) {
        e = hipEventCreateWithFlags(&b->ev[c], hipEventDisableTiming);
        if (e != hipSuccess) st = fail_hip(e, "hipEventCreate");
      }
    }
  }
  if (!st) st = build_batch(b, nullptr, nullptr, nullptr);
  if (!st && b->use_graph) {
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
      st = fail_hip(e, "hipStreamCreate");
    } else {
      st = capture(b->fwd_seq, cs, &b->gf, &b->ef);
      if (!st) st = capture(b->adj_seq, cs, &b->ga, &b->ea);
      (void)hipStreamDestroy(cs);
    }
  }
  (void)stream;
  if (st) {
    delete b;
    return st;
  }
  {
    std::lock_guard<std::mutex> lk(g_registry_mu);
    g_batches.insert(b);
    for (pc_plan p : b->plans) ++p->batch_refs;
  }
  *out = b;
  return PC_SUCCESS;
}

namespace {

// Every input and output of a batch call non-null; an instance's output
// overlaps neither another output nor any input (inputs may overlap each
// other: they are only read).
pc_status check_batch_buffers(pc_batch b, const float* const* inputs, float* const* outputs) {
  if (!inputs || !outputs) return fail(PC_ERROR_INVALID_VALUE, "null input or output array");
  struct Span {
    uintptr_t a, e;
    size_t i;
  };
  std::vector<Span> outs, ins;
  for (size_t i = 0; i < b->plans.size(); ++i) {
    if (!inputs[i] || !outputs[i]) return fail(PC_ERROR_INVALID_VALUE, "null buffer for instance " + std::to_string(i));
    const size_t bytes = (size_t)(b->plans[i]->d.batch * b->plans[i]->n_total) * sizeof(float);
    outs.push_back({reinterpret_cast<uintptr_t>(outputs[i]), reinterpret_cast<uintptr_t>(outputs[i]) + bytes, i});
    ins.push_back({reinterpret_cast<uintptr_t>(inputs[i]), reinterpret_cast<uintptr_t>(inputs[i]) + bytes, i});
  }
  std::sort(outs.begin(), outs.end(), [](const Span& x, const Span& y) { return x.a < y.a; });
  for (size_t k = 1; k < outs.size(); ++k)
    if (outs[k].a < outs[k - 1].e)
      return fail(PC_ERROR_INVALID_VALUE, "outputs of instances " + std::to_string(outs[k - 1].i) + " and " +
                                              std::to_string(outs[k].i) + " overlap");
  for (const Span& x : ins) {
    // the first output starting at or after x.a, and the one before it
    auto it = std::lower_bound(outs.begin(), outs.end(), x.a, [](const Span& o, uintptr_t v) { return o.a < v; });
    if ((it != outs.end() && it->a < x.e) || (it != outs.begin() && std::prev(it)->e > x.a))
      return fail(PC_ERROR_INVALID_VALUE, "input of instance " + std::to_string(x.i) + " overlaps an output");
  }
  return PC_SUCCESS;
}

}  // namespace

static pc_status batch_run(pc_batch b, bool adjoint, const float* const* inputs, float* const* outputs,
                           void* stream) {
  pc_status st = check_batch(b);
  if (st) return st;
  if ((st = check_batch_buffers(b, inputs, outputs))) return st;
  DeviceGuard g(b->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int c = adjoint ? 1 : 0;
  const size_t n = b->plans.size();
  std::vector<float*> cur(2 * n);
  for (size_t i = 0; i < n; ++i) {
    cur[2 * i] = const_cast<float*>(inputs[i]);  // read only: the kernels take it as const
    cur[2 * i + 1] = outputs[i];
  }
  for (pc_plan p : b->plans) p->saved_state = 0;  // the batch uses the plans' workspaces
  if (cur != b->last[c]) {
    // the staging slot is rewritten only once its previous upload has run
    hipError_t e = hipEventSynchronize(b->ev[c]);
    if (e != hipSuccess) return fail_hip(e, "hipEventSynchronize");
    std::copy(cur.begin(), cur.end(), b->htab + c * 2 * n);
    e = hipMemcpyAsync(b->dtab + c * 2 * n, b->htab + c * 2 * n, 2 * n * sizeof(float*), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(b->ev[c], s);
    if (e != hipSuccess) {
      b->last[c].clear();
      return fail_hip(e, "batch pointer upload");
    }
    b->last[c] = cur;
  }
  if (!b->use_graph) return run_seq(adjoint ? b->adj_seq : b->fwd_seq, s);
  hipError_t e = hipGraphLaunch(adjoint ? b->ea : b->ef, s);
  if (e != hipSuccess) return fail_hip(e, "hipGraphLaunch");
  return PC_SUCCESS;
}

pc_status pc_batch_apply(pc_batch b, const float* const* inputs, float* const* outputs, void* stream) {
  return batch_run(b, false, inputs, outputs, stream);
}
pc_status pc_batch_apply_adjoint(pc_batch b, const float* const* inputs, float* const* outputs, void* stream) {
  return batch_run(b, true, inputs, outputs, stream);
}

pc_status pc_batch_destroy(pc_batch b) {
  {
    std::lock_guard<std::mutex> lk(g_registry_mu);
    if (!b || !g_batches.count(b)) return fail(PC_ERROR_INVALID_VALUE, "batch handle is not a live batch");
    g_batches.erase(b);
    for (pc_plan p : b->plans) --p->batch_refs;
  }
  DeviceGuard g(b->device);
  hipError_t e = hipDeviceSynchronize();
  delete b;
  if (e != hipSuccess) return fail_hip(e, "hipDeviceSynchronize before free");
  return PC_SUCCESS;
}

const char* pc_status_string(pc_status st) {
  switch (st) {
    case PC_SUCCESS: return "PC_SUCCESS";
    case PC_ERROR_INVALID_VALUE: return "PC_ERROR_INVALID_VALUE";
    case PC_ERROR_UNSUPPORTED: return "PC_ERROR_UNSUPPORTED";
    case PC_ERROR_OUT_OF_MEMORY: return "PC_ERROR_OUT_OF_MEMORY";
    case PC_ERROR_HIP: return "PC_ERROR_HIP";
    case PC_ERROR_INVALID_PLAN: return "PC_ERROR_INVALID_PLAN";
  }
  return "PC_UNKNOWN_STATUS";
}

const char* pc_last_error(void) { return g_last_error.c_str(); }

pc_status pc_tune_set(const pc_tune_entry* entries, int32_t count) {
  if (count < 0 || (count > 0 && !entries)) return fail(PC_ERROR_INVALID_VALUE, "null entries or negative count");
  std::vector<pc::TuneEntry> t;
  for (int32_t i = 0; i < count; ++i) {
    const pc_tune_entry& e = entries[i];
    if (e.knob < PC_TUNE_COLS_FWD_LATE || e.knob > PC_TUNE_KEEP)
      return fail(PC_ERROR_INVALID_VALUE, "unknown knob " + std::to_string(e.knob) + " in entry " + std::to_string(i));
    t.push_back({e.key, e.knob, e.length, e.value});
  }
  pc::tune_set(t);
  return PC_SUCCESS;
}

pc_status pc_tune_key(const pc_plan_desc* desc, uint64_t* key) {
  if (!desc || !key) return fail(PC_ERROR_INVALID_VALUE, "null argument");
  *key = pc::tune_key(*desc);
  return PC_SUCCESS;
}

pc_status pc_tune_batch_key(int32_t count, const pc_plan* plans, uint64_t* key) {
  if (count < 1 || !plans || !key) return fail(PC_ERROR_INVALID_VALUE, "null argument or count < 1");
  std::vector<pc_plan_desc> ds;
  for (int32_t i = 0; i < count; ++i) {
    pc_status st = check_plan(plans[i]);
    if (st) return st;
    ds.push_back(plans[i]->d);
  }
  *key = pc::tune_batch_key(ds);
  return PC_SUCCESS;
}

pc_status pc_plan_create(pc_plan* out, const pc_plan_desc* desc, const float* windows, const float* h,
                         void* stream) {
  if (!out) return fail(PC_ERROR_INVALID_VALUE, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(PC_ERROR_INVALID_VALUE, "desc is NULL");
  if (!windows || !h) return fail(PC_ERROR_INVALID_VALUE, "windows or h is NULL");
  pc_plan_s* p = nullptr;
  pc_status st = create_plan(*desc, windows, h, static_cast<hipStream_t>(stream), &p);
  if (st) return st;
  {
    std::lock_guard<std::mutex> g(g_registry_mu);
    g_registry.insert(p);
  }
  *out = p;
  return PC_SUCCESS;
}

// The forward of a convolution-product 2D plan leaves the row transforms of
// the windowed input in the workspace (and, kept, U_k).
static void remember(pc_plan p, const float* u, int64_t batch, int state) {
  p->saved_u = u;
  p->saved_batch = batch;
  p->saved_state = (p->pconv || p->path < 2) ? 0 : state;
}

pc_status pc_apply(pc_plan p, const float* u, float* y, int64_t batch, void* stream) {
  pc_status st = check_apply(p, u, y, batch);
  if (st || batch == 0) return st;
  DeviceGuard g(p->device);
  hipError_t e = p->pconv ? run_adjoint(p, u, y, batch, static_cast<hipStream_t>(stream))
                          : run_forward(p, u, y, batch, static_cast<hipStream_t>(stream));
  remember(p, u, batch, e == hipSuccess ? 1 : 0);
  if (e != hipSuccess) return fail_hip(e, "pc_apply launch");
  return PC_SUCCESS;
}

pc_status pc_apply_save(pc_plan p, const float* u, float* y, int64_t batch, void* stream) {
  pc_status st = check_apply(p, u, y, batch);
  if (st || batch == 0) return st;
  DeviceGuard g(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  int state = 1;
  if (p->pconv || p->path < 2) {
    e = p->pconv ? run_adjoint(p, u, y, batch, s) : run_forward(p, u, y, batch, s);
  } else if (p->path == 2) {
    e = pc::launch_fwd2d(p->p2, u, y, batch, s, p->tr(), true);
    if (p->p2.keep) state = 2;
  } else if (p->sec_batch_keep) {
    e = launch_seq(p->sec_batch_keep->fwd_seq, s, p->tr(), u, batch);
    if (e == hipSuccess) e = pc::launch_sec_scatter(p->sec, y, false, batch, s, p->tr());
    state = 2;
  } else {
    e = run_sections(p, u, y, batch, false, s);
  }
  remember(p, u, batch, e == hipSuccess ? state : 0);
  if (e != hipSuccess) return fail_hip(e, "pc_apply_save launch");
  return PC_SUCCESS;
}

pc_status pc_apply_adjoint(pc_plan p, const float* v, float* x, int64_t batch, void* stream) {
  pc_status st = check_apply(p, v, x, batch);
  if (st || batch == 0) return st;
  DeviceGuard g(p->device);
  p->saved_state = 0;  // the adjoint's planes overwrite the workspace
  hipError_t e = p->pconv ? run_forward(p, v, x, batch, static_cast<hipStream_t>(stream))
                          : run_adjoint(p, v, x, batch, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail_hip(e, "pc_apply_adjoint launch");
  return PC_SUCCESS;
}

pc_status pc_destroy(pc_plan p) {
  {
    std::lock_guard<std::mutex> g(g_registry_mu);
    if (!p || !g_registry.count(p)) return fail(PC_ERROR_INVALID_PLAN, "plan handle is not a live plan");
    if (p->batch_refs > 0)
      return fail(PC_ERROR_INVALID_VALUE, "the plan is held by " + std::to_string(p->batch_refs) +
                                              " live batch(es); destroy them first");
    g_registry.erase(p);
  }
  DeviceGuard g(p->device);
  hipError_t e = hipDeviceSynchronize();
  delete p;
  if (e != hipSuccess) return fail_hip(e, "hipDeviceSynchronize before free");
  return PC_SUCCESS;
}

pc_status pc_plan_query(pc_plan p, pc_plan_info* info) {
  pc_status st = check_plan(p);
  if (st) return st;
  if (!info) return fail(PC_ERROR_INVALID_VALUE, "info is NULL");
  pc_plan_info r{};
  r.path = p->path;
  if (p->path == 0) {
    r.fft_inner = p->s1.L;
    r.fft_outer = 1;
  } else if (p->path == 1) {
    r.fft_inner = p->l1.L;
    r.fft_outer = p->l1.R;
    r.n_items = p->l1.n_items;
  } else if (p->path == 2) {
    r.fft_inner = p->p2.N1;
    r.fft_outer = p->p2.N2;
  } else {
    for (pc_plan_s* q : p->sec_sub) {
      r.fft_inner = std::max(r.fft_inner, (int32_t)q->d.n0);
      r.fft_outer = std::max(r.fft_outer, (int32_t)q->d.n1);
    }
    r.n_items = p->sec.n_sec;
  }
  r.spectra_bytes = p->spectra_bytes;
  r.window_bytes = p->window_bytes;
  r.workspace_bytes = p->workspace_bytes;
  r.keep_bytes = p->keep_bytes;
  r.spectra_count = p->spec_count;
  *info = r;
  return PC_SUCCESS;
}

pc_status pc_plan_set_spectra(pc_plan p, const void* spec, void* stream) {
  pc_status st = check_plan(p);
  if (st) return st;
  if (!spec) return fail(PC_ERROR_INVALID_VALUE, "spec is NULL");
  if (p->path == 3 && p->pconv)
    return fail(PC_ERROR_UNSUPPORTED, "sectioned product-convolution plans do not import spectra "
                                      "(create the plan with PC_PLAN_FULL_GRID)");
  DeviceGuard g(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->path == 3) {
    hipError_t e = pc::launch_transpose_set(p->tr_spec, const_cast<float2*>(static_cast<const float2*>(spec)), true, s);
    if (e != hipSuccess) return fail_hip(e, "pc_plan_set_spectra launch");
    return PC_SUCCESS;
  }
  const float2* in = static_cast<const float2*>(spec);
  hipError_t e;
  if (p->pconv) {  // the plan stores the spectra of the flipped responses
    e = pc::launch_conj(in, p->conj_ws, p->spec_count, s);
    if (e != hipSuccess) return fail_hip(e, "pc_plan_set_spectra launch");
    in = p->conj_ws;
  }
  if (p->path == 0)
    e = pc::launch_spectra1d(&p->s1, nullptr, in, nullptr, true, s);
  else if (p->path == 1)
    e = pc::launch_spectra1d(nullptr, &p->l1, in, nullptr, true, s);
  else
    e = pc::launch_spectra2d(p->p2, in, nullptr, true, s);
  if (e != hipSuccess) return fail_hip(e, "pc_plan_set_spectra launch");
  return PC_SUCCESS;
}

pc_status pc_plan_get_spectra(pc_plan p, void* spec, void* stream) {
  pc_status st = check_plan(p);
  if (st) return st;
  if (!spec) return fail(PC_ERROR_INVALID_VALUE, "spec is NULL");
  DeviceGuard g(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  float2* out = static_cast<float2*>(spec);
  hipError_t e;
  if (p->path == 3)
    e = pc::launch_transpose_set(p->tr_spec, out, false, s);
  else if (p->path == 0)
    e = pc::launch_spectra1d(&p->s1, nullptr, nullptr, out, false, s);
  else if (p->path == 1)
    e = pc::launch_spectra1d(nullptr, &p->l1, nullptr, out, false, s);
  else
    e = pc::launch_spectra2d(p->p2, nullptr, out, false, s);
  if (e == hipSuccess && p->pconv) e = pc::launch_conj(out, out, p->spec_count, s);
  if (e != hipSuccess) return fail_hip(e, "pc_plan_get_spectra launch");
  return PC_SUCCESS;
}

static hipError_t run_grad_spectra(pc_plan p, const float* u, const float* gy, float2* out, int64_t batch,
                                   bool rows_u, const float2* keep, hipStream_t s) {
  // product-convolution: sum_b conj(F^* u_b) F^*(w_k . gy_b) is the
  // conjugate of the convolution-product sum with u and gy exchanged
  const float* a = p->pconv ? gy : u;
  const float* b = p->pconv ? u : gy;
  hipError_t e;
  if (p->path == 0)
    e = pc::launch_grad1d_small(p->s1, a, b, out, batch, p->grad_ws, s, p->tr());
  else if (p->path == 1)
    e = pc::launch_grad1d_large(p->l1, a, b, out, batch, p->grad_ws, s, p->tr());
  else if (p->path == 2)
    e = pc::launch_grad2d(p->p2, a, b, out, batch, p->grad_ws, s, p->tr(), rows_u || p->pconv, p->pconv ? nullptr : keep);
  else
    e = run_sec_backward(p, u, gy, nullptr, out, batch, rows_u ? 0 : 1, s);
  if (e == hipSuccess && p->pconv) e = pc::launch_conj(out, out, p->spec_count, s);
  return e;
}

static bool has_gradients(pc_plan p) { return (p->d.flags & PC_PLAN_GRADIENTS) != 0; }

pc_status pc_backward(pc_plan p, const float* u, const float* gy, float* gu, void* gspec, int64_t batch,
                      int32_t use_saved, void* stream) {
  pc_status st = check_plan(p);
  if (st) return st;
  if (batch < 1 || batch > p->d.batch)
    return fail(PC_ERROR_INVALID_VALUE, "batch " + std::to_string(batch) + " outside [1, " +
                                            std::to_string(p->d.batch) + "]");
  if (!u || !gy || (!gu && !gspec)) return fail(PC_ERROR_INVALID_VALUE, "null pointer");
  if (gspec && !has_gradients(p)) return fail(PC_ERROR_INVALID_VALUE, "plan was created without PC_PLAN_GRADIENTS");
  const size_t bytes = (size_t)(batch * p->n_total) * sizeof(float);
  if (gu && (overlaps(gy, gu, bytes) || overlaps(u, gu, bytes)))
    return fail(PC_ERROR_INVALID_VALUE, "gu overlaps u or gy");
  DeviceGuard g(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  float2* gs = static_cast<float2*>(gspec);
  const int state = (use_saved && p->saved_u == u && p->saved_batch == batch) ? p->saved_state : 0;
  hipError_t e = hipSuccess;
  if (p->path == 3) {
    if (gspec)
      e = run_sec_backward(p, u, gy, gu, gs, batch, state, s);
    else
      e = p->pconv ? run_forward(p, gy, gu, batch, s) : run_adjoint(p, gy, gu, batch, s);
  } else if (p->path == 2 && !p->pconv && gspec && !p->p2.adj_fused) {
    // the gradient pass leaves V = colFFT(rowFFT(gy)) for the adjoint's
    // column pass, and uses the row transforms or U_k the forward left
    e = pc::launch_grad2d(p->p2, u, gy, gs, batch, p->grad_ws, s, p->tr(), state == 0,
                          state == 2 ? p->p2.keep : nullptr);
    if (e == hipSuccess && gu) e = pc::launch_adj2d_tail(p->p2, gu, batch, s, p->tr());
  } else {
    if (gspec) e = run_grad_spectra(p, u, gy, gs, batch, true, nullptr, s);
    if (e == hipSuccess && gu) e = p->pconv ? run_forward(p, gy, gu, batch, s) : run_adjoint(p, gy, gu, batch, s);
  }
  if (gu || p->path < 2 || p->pconv)
    p->saved_state = 0;
  else  // the gradient left (or recomputed) the row transforms of u
    remember(p, u, batch, std::max(state, 1));
  if (e != hipSuccess) return fail_hip(e, "pc_backward launch");
  return PC_SUCCESS;
}

pc_status pc_plan_set_budget(pc_plan p, int64_t bytes) {
  pc_status st = check_plan(p);
  if (st) return st;
  if (bytes < 0) return fail(PC_ERROR_INVALID_VALUE, "budget must be >= 0");
  DeviceGuard g(p->device);
  return set_keep(p, bytes);
}

pc_status pc_plan_sections(pc_plan p, pc_section_info* info, int32_t capacity, int32_t* count) {
  pc_status st = check_plan(p);
  if (st) return st;
  if (!count || (!info && capacity > 0) || capacity < 0) return fail(PC_ERROR_INVALID_VALUE, "null count or info");
  const int n = p->path == 3 ? (int)p->sec_geom.size() : 0;
  *count = n;
  int64_t off = 0;
  for (int i = 0; i < n && i < capacity; ++i) {
    const std::array<int64_t, 10>& gm = p->sec_geom[(size_t)i];
    pc_section_info r{};
    r.term = p->sec_k[(size_t)i];
    r.win_o1 = gm[0]; r.win_p1 = gm[1]; r.win_o2 = gm[2]; r.win_p2 = gm[3];
    r.lag_o1 = gm[4]; r.lag_q1 = gm[5]; r.lag_o2 = gm[6]; r.lag_q2 = gm[7];
    r.m1 = gm[8]; r.m2 = gm[9];
    r.spec_offset = off;
    off += gm[8] * (gm[9] / 2 + 1);
    info[i] = r;
  }
  return PC_SUCCESS;
}

pc_status pc_grad_spectra(pc_plan p, const float* u, const float* gy, void* gspec, int64_t batch, void* stream) {
  pc_status st = check_plan(p);
  if (st) return st;
  if (!has_gradients(p)) return fail(PC_ERROR_INVALID_VALUE, "plan was created without PC_PLAN_GRADIENTS");
  if (batch < 1 || batch > p->d.batch)
    return fail(PC_ERROR_INVALID_VALUE, "batch " + std::to_string(batch) + " outside [1, " +
                                            std::to_string(p->d.batch) + "]");
  if (!u || !gy || !gspec) return fail(PC_ERROR_INVALID_VALUE, "null pointer");
  DeviceGuard g(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = run_grad_spectra(p, u, gy, static_cast<float2*>(gspec), batch, true, nullptr, s);
  // the 2D gradient recomputed the row transforms of u into the workspace
  remember(p, u, batch, e == hipSuccess ? 1 : 0);
  if (e != hipSuccess) return fail_hip(e, "pc_grad_spectra launch");
  return PC_SUCCESS;
}

pc_status pc_plan_set_responses(pc_plan p, const float* h, void* stream) {
  pc_status st = check_plan(p);
  if (st) return st;
  if (!h) return fail(PC_ERROR_INVALID_VALUE, "h is NULL");
  if (p->path == 3)
    return fail(PC_ERROR_UNSUPPORTED, "sectioned plans are built for the supports of their responses "
                                      "(create the plan with PC_PLAN_FULL_GRID)");
  DeviceGuard g(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (p->pconv) {  // the plan holds the operator of the flipped responses
    float* fl = reinterpret_cast<float*>(p->conj_ws);
    e = pc::launch_flip(h, fl, p->d.m, p->d.n0, p->d.n1, s);
    h = fl;
  }
  if (e == hipSuccess) {
    if (p->path == 0) {
      e = pc::launch_spec1d_full(p->s1.L, h, const_cast<float2*>(p->s1.H), p->d.m, p->s1.tw, s);
    } else if (p->path == 1) {
      float2* Hd = const_cast<float2*>(p->l1.Hd);
      e = pc::launch_fold_fft(p->l1, h, p->d.m, Hd, false, s);
      if (e == hipSuccess) e = pc::launch_origin_phase1d(p->l1, Hd, s);
    } else {
      e = pc::launch_spec2d(p->p2, h, s);
    }
  }
  if (e != hipSuccess) return fail_hip(e, "pc_plan_set_responses launch");
  return PC_SUCCESS;
}

pc_status pc_construct_project(int64_t n, int32_t m, int64_t rows, const float* tvir, const int64_t* lags,
                               const float* windows, float* h, void* stream) {
  pc_status st = check_construct(n, m, rows, tvir, windows, h, lags);
  if (st) return st;
  if ((reinterpret_cast<uintptr_t>(tvir) | reinterpret_cast<uintptr_t>(windows)) % 16)
    return fail(PC_ERROR_INVALID_VALUE, "tvir and windows must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int splits = pc::gemm_splits(n);
  CallTemps t;
  float *part = nullptr, *gpart = nullptr;
  double *rhs = nullptr, *work = nullptr, *G = nullptr;
  int64_t* dl = nullptr;
  int* dfail = nullptr;
  if ((st = t.alloc(&part, (size_t)splits * rows * m)) || (st = t.alloc(&gpart, (size_t)splits * m * m)) ||
      (st = t.alloc(&rhs, (size_t)rows * m)) || (st = t.alloc(&work, (size_t)rows * m)) ||
      (st = t.alloc(&G, (size_t)m * m)) || (st = t.alloc(&dfail, 1)) || (st = t.upload(&dl, lags, (size_t)rows)) ||
      (st = t.commit(s)))
    return st;
  hipError_t e = pc::launch_fill_zero(h, (int64_t)m * n, s);
  // right-hand sides W T(x, .)^T for every row, and the Gram matrix W W^T
  if (e == hipSuccess) e = pc::launch_gemm_nt(tvir, rows, windows, m, n, part, s);
  if (e == hipSuccess) e = pc::launch_sum_splits(part, splits, rows * m, rhs, s);
  if (e == hipSuccess) e = pc::launch_gemm_nt(windows, m, windows, m, n, gpart, s);
  if (e == hipSuccess) e = pc::launch_sum_splits(gpart, splits, (int64_t)m * m, G, s);
  if (e == hipSuccess) e = pc::launch_cholesky(G, m, dfail, s);
  if (e == hipSuccess) e = pc::launch_row_solve(false, G, nullptr, m, rhs, work, rows, dl, n, h, s);
  if (e != hipSuccess) return fail_hip(e, "pc_construct_project launch");
  return finish_construct(s, dfail, "pc_construct_project");
}

pc_status pc_construct_interpolate(int64_t n, int32_t m, int64_t rows, const float* samples, const int64_t* lags,
                                   const int64_t* nodes, const float* windows, float* h, void* stream) {
  pc_status st = check_construct(n, m, rows, samples, windows, h, lags);
  if (st) return st;
  if (!nodes) return fail(PC_ERROR_INVALID_VALUE, "nodes is NULL");
  {
    std::vector<char> seen((size_t)n, 0);
    for (int i = 0; i < m; ++i) {
      if (nodes[i] < 0 || nodes[i] >= n || seen[(size_t)nodes[i]])
        return fail(PC_ERROR_INVALID_VALUE, "nodes must be distinct and in [0, n)");
      seen[(size_t)nodes[i]] = 1;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallTemps t;
  double *src = nullptr, *work = nullptr, *E = nullptr;
  int64_t *dl = nullptr, *dn = nullptr;
  int *perm = nullptr, *dfail = nullptr;
  if ((st = t.alloc(&src, (size_t)rows * m)) || (st = t.alloc(&work, (size_t)rows * m)) ||
      (st = t.alloc(&E, (size_t)m * m)) || (st = t.alloc(&perm, (size_t)m)) || (st = t.alloc(&dfail, 1)) ||
      (st = t.upload(&dl, lags, (size_t)rows)) || (st = t.upload(&dn, nodes, (size_t)m)) || (st = t.commit(s)))
    return st;
  hipError_t e = pc::launch_fill_zero(h, (int64_t)m * n, s);
  if (e == hipSuccess) e = pc::launch_node_matrix(windows, m, n, dn, E, s);
  if (e == hipSuccess) e = pc::launch_lu(E, m, perm, dfail, s);
  if (e == hipSuccess) e = pc::launch_to_double(samples, rows * m, src, s);
  if (e == hipSuccess) e = pc::launch_row_solve(true, E, perm, m, src, work, rows, dl, n, h, s);
  if (e != hipSuccess) return fail_hip(e, "pc_construct_interpolate launch");
  return finish_construct(s, dfail, "pc_construct_interpolate");
}

pc_status pc_wavelet_transform(int32_t inverse, int64_t n, int32_t levels, int32_t taps, const float* lowpass,
                               int64_t count, int64_t stride, int64_t dist, const float* in, float* out,
                               void* stream) {
  pc::WaveletFilter f;
  pc_status st = make_filter(taps, lowpass, f);
  if (st) return st;
  if (!is_pow2(n) || n < 2) return fail(PC_ERROR_INVALID_VALUE, "n must be a power of two >= 2");
  if (levels < 0 || levels > 62 || (n >> levels) < 1) return fail(PC_ERROR_INVALID_VALUE, "levels out of range");
  if (count < 1 || stride < 1 || dist < 1) return fail(PC_ERROR_INVALID_VALUE, "count, stride, dist must be >= 1");
  if (!in || !out || in == out) return fail(PC_ERROR_INVALID_VALUE, "null or identical in/out");
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallTemps t;
  float *s1 = nullptr, *s2 = nullptr;
  if ((st = t.alloc(&s1, (size_t)(count * (n / 2 + 1)))) || (st = t.alloc(&s2, (size_t)(count * (n / 2 + 1)))) ||
      (st = t.commit(s)))
    return st;
  hipError_t e = pc::launch_wavelet(inverse != 0, n, levels, f, count, stride, dist, in, out, s1, s2, s);
  if (e != hipSuccess) return fail_hip(e, "pc_wavelet_transform launch");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e, "pc_wavelet_transform");
  return PC_SUCCESS;
}

pc_status pc_wavelet_transform_noalloc(int32_t inverse, int64_t n, int32_t levels, int32_t taps,
                                       const float* lowpass, int64_t count, int64_t stride, int64_t dist,
                                       const float* in, float* out, void* stream) {
  pc::WaveletFilter f;
  pc_status st = make_filter(taps, lowpass, f);
  if (st) return st;
  if (!is_pow2(n) || n < 2) return fail(PC_ERROR_INVALID_VALUE, "n must be a power of two >= 2");
  if (levels < 0 || levels > 62 || (n >> levels) < 1) return fail(PC_ERROR_INVALID_VALUE, "levels out of range");
  if (count < 1 || stride < 1 || dist < 1) return fail(PC_ERROR_INVALID_VALUE, "count, stride, dist must be >= 1");
  if (!in || !out || in == out) return fail(PC_ERROR_INVALID_VALUE, "null or identical in/out");
  if (count > pc::WAVELET_STATIC_FLOATS / n)
    return fail(PC_ERROR_INVALID_VALUE, "count * n = " + std::to_string(count) + " * " + std::to_string(n) +
                                            " exceeds the fixed scratch (" +
                                            std::to_string(pc::WAVELET_STATIC_FLOATS) + " samples per call)");
  hipError_t e = pc::launch_wavelet_static(inverse != 0, n, levels, f, count, stride, dist, in, out,
                                           static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail_hip(e, "pc_wavelet_transform_noalloc launch");
  return PC_SUCCESS;
}

pc_status pc_plan_create_meyer(pc_plan* out, int64_t n, int32_t levels, int32_t taps, const float* lowpass,
                               int64_t count, const int64_t* lam, const int64_t* mu, const float* c, int64_t batch,
                               uint32_t flags, void* stream) {
  if (!out) return fail(PC_ERROR_INVALID_VALUE, "out is NULL");
  *out = nullptr;
  pc::WaveletFilter f;
  pc_status st = make_filter(taps, lowpass, f);
  if (st) return st;
  if (!is_pow2(n)) return fail(PC_ERROR_INVALID_VALUE, "n must be a power of two");
  if (levels < 0 || levels > 62 || (n >> levels) < 1) return fail(PC_ERROR_INVALID_VALUE, "levels out of range");
  if (count < 1 || !lam || !mu || !c) return fail(PC_ERROR_INVALID_VALUE, "empty or null coefficient list");
  std::vector<int64_t> mus(mu, mu + count);
  for (int64_t i = 0; i < count; ++i)
    if (lam[i] < 0 || lam[i] >= n || mu[i] < 0 || mu[i] >= n)
      return fail(PC_ERROR_INVALID_VALUE, "coefficient indices must be in [0, n)");
  std::sort(mus.begin(), mus.end());
  mus.erase(std::unique(mus.begin(), mus.end()), mus.end());
  const int64_t m2 = (int64_t)mus.size();
  if (m2 > INT32_MAX) return fail(PC_ERROR_INVALID_VALUE, "too many terms");
  // rows 0..m2-1: unit vectors e_mu (-> windows psi_mu); rows m2..2m2-1: the
  // coefficient columns c_{., mu} (-> c~_mu), both synthesised on the device
  std::vector<float> coef((size_t)(2 * m2 * n), 0.f);
  for (int64_t i = 0; i < m2; ++i) coef[(size_t)(i * n + mus[(size_t)i])] = 1.f;
  for (int64_t i = 0; i < count; ++i) {
    const int64_t r = std::lower_bound(mus.begin(), mus.end(), mu[i]) - mus.begin();
    coef[(size_t)((m2 + r) * n + lam[i])] += c[i];
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<float> syn(coef.size());
  {
    CallTemps t;
    float *din = nullptr, *dout = nullptr, *s1 = nullptr, *s2 = nullptr;
    if ((st = t.upload(&din, coef.data(), coef.size())) || (st = t.alloc(&dout, coef.size())) ||
        (st = t.alloc(&s1, (size_t)(2 * m2 * (n / 2 + 1)))) || (st = t.alloc(&s2, (size_t)(2 * m2 * (n / 2 + 1)))) ||
        (st = t.commit(s)))
      return st;
    hipError_t e = pc::launch_wavelet(true, n, levels, f, 2 * m2, 1, n, din, dout, s1, s2, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(syn.data(), dout, syn.size() * sizeof(float), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail_hip(e, "Meyer synthesis");
  }
  // responses carry the grid's quadrature weight 1/n
  const float inv_n = 1.0f / (float)n;
  for (size_t i = (size_t)(m2 * n); i < syn.size(); ++i) syn[i] *= inv_n;
  pc_plan_desc d{};
  d.ndim = 1;
  d.m = (int32_t)m2;
  d.n0 = n;
  d.n1 = 1;
  d.batch = batch;
  d.w_format = PC_W_DENSE;
  d.flags = flags;
  pc_plan_s* p = nullptr;
  if ((st = create_plan(d, syn.data(), syn.data() + m2 * n, s, &p))) return st;
  {
    std::lock_guard<std::mutex> g(g_registry_mu);
    g_registry.insert(p);
  }
  *out = p;
  return PC_SUCCESS;
}

pc_status pc_plan_set_tracing(pc_plan p, int32_t enable) {
  pc_status st = check_plan(p);
  if (st) return st;
  p->tracing = enable != 0;
  return PC_SUCCESS;
}

pc_status pc_plan_trace_stats(pc_plan p, pc_kernel_stat* stats, int32_t capacity, int32_t* count) {
  pc_status st = check_plan(p);
  if (st) return st;
  if (!count || (capacity > 0 && !stats)) return fail(PC_ERROR_INVALID_VALUE, "null output pointer");
  DeviceGuard g(p->device);
  hipError_t e = p->tracer.flush();
  if (e != hipSuccess) return fail_hip(e, "trace events");
  const int32_t n = (int32_t)p->tracer.stats.size();
  for (int32_t i = 0; i < n && i < capacity; ++i) {
    const auto& x = p->tracer.stats[i];
    pc_kernel_stat r{};
    std::snprintf(r.kernel, sizeof(r.kernel), "%s", x.name.c_str());
    r.launches = x.n;
    r.total_ms = x.tot;
    r.min_ms = x.mn;
    r.max_ms = x.mx;
    stats[i] = r;
  }
  *count = n;
  return PC_SUCCESS;
}

pc_status pc_plan_trace_reset(pc_plan p) {
  pc_status st = check_plan(p);
  if (st) return st;
  DeviceGuard g(p->device);
  hipError_t e = p->tracer.flush();
  p->tracer.stats.clear();
  if (e != hipSuccess) return fail_hip(e, "trace events");
  return PC_SUCCESS;
}

}  // extern "C"
