// 1D kernels of the convolution-product expansion (eq. 1.4 and its adjoint).
//
// Real signals are processed two at a time as one complex signal
// (u_a + i u_b): windows and impulse responses are real, so
// H_m (u_a + i u_b) = H_m u_a + i H_m u_b exactly, and one complex FFT serves
// two outputs.  The identity of section 3.5 is applied once per output:
// since the DFT is linear, sum_k F(H_k . U_k) = F(sum_k H_k . U_k), so the
// forward pass pays m forward transforms and one inverse transform, and the
// adjoint pass one forward and m inverse transforms.
#include "fft_engine.hpp"
#include "pc_internal.hpp"

namespace pc {

#define PC_FOR_EACH_L(X) \
  X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192) \
  X(96) X(192) X(384) X(768) X(1536) X(3072) X(6144)

bool fft_size_supported(int64_t L) {
  switch (L) {
#define PC_CASE(LL) case LL:
    PC_FOR_EACH_L(PC_CASE)
#undef PC_CASE
    return true;
    default:
      return false;
  }
}

// ===========================================================================
// N <= 8192: one workgroup (or one slice of it) per signal pair
// ===========================================================================

// Small batches (fewer workgroups than compute units) run split: the NF
// transform slots of a workgroup share one pair and take its terms in turn,
// and their spectral sums are added in LDS before the slot-0 result is kept.
// Sum of the slots' acc into slot 0's acc (every thread calls it).
template <int L, int P, int NF>
__device__ __forceinline__ void sum_slots(float2 (&acc)[P], float2* lds, int c, int t) {
  constexpr int T = L / P;
  __syncthreads();  // every slot's transforms are done with LDS
#pragma unroll
  for (int e = 0; e < P; ++e) lds[c * lds_len<L>() + lpad(t + T * e)] = acc[e];
  __syncthreads();
  if (c == 0) {
    for (int sl = 1; sl < NF; ++sl) {
#pragma unroll
      for (int e = 0; e < P; ++e) acc[e] = cadd(acc[e], lds[sl * lds_len<L>() + lpad(t + T * e)]);
    }
  }
  // the next transform's first LDS write follows a barrier of its own
}

// Plan-time spectra H_k = F^* h_k (full complex, natural order).
template <int L>
__global__ __launch_bounds__(ffts_per_block(L) * fft_threads(L)) void k_spec1d_full(
    const float* __restrict__ h, float2* __restrict__ H, int m, const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(L), T = L / P, NF = ffts_per_block(L);
  __shared__ float2 lds[NF * lds_len<L>()];
  __shared__ float2 twl[L];
  stage_twiddles<L>(twl, tw);
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int k = blockIdx.x * NF + c;
  const bool ok = k < m;
  float2 v[P];
#pragma unroll
  for (int e = 0; e < P; ++e) v[e] = make_float2(ok ? h[(int64_t)k * L + t + T * e] : 0.f, 0.f);
  fft_wg<L, P, false>(v, lds + c * lds_len<L>(), twl, t);
  if (ok) {
#pragma unroll
    for (int e = 0; e < P; ++e) H[(int64_t)k * L + t + T * e] = v[e];
  }
}

// y = H_m u for signal pairs.
template <int L>
__global__ __launch_bounds__(ffts_per_block(L) * fft_threads(L)) void k_fwd1d_small(
    const float* __restrict__ u, float* __restrict__ y, int64_t batch, int m, const float* __restrict__ w,
    const float2* __restrict__ H, const float2* __restrict__ tw, int split) {
  constexpr int P = points_per_thread(L), T = L / P, NF = ffts_per_block(L);
  __shared__ float2 lds[NF * lds_len<L>()];
  __shared__ float2 twl[L];
  stage_twiddles<L>(twl, tw);
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int64_t pair = split ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * NF + c;
  const int64_t sa = 2 * pair, sb = sa + 1;
  const bool keep = !split || c == 0;
  const bool va = sa < batch, vb = sb < batch;
  float ua[P], ub[P];
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int n = t + T * e;
    ua[e] = va ? u[sa * L + n] : 0.f;
    ub[e] = vb ? u[sb * L + n] : 0.f;
  }
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  float2* my = lds + c * lds_len<L>();
  // every slot makes the same number of transform calls (they hold barriers):
  // a slot past the last term transforms a valid term with zero weight
  const int nk = split ? (m + NF - 1) / NF : m;
  for (int i = 0; i < nk; ++i) {
    const int kt = split ? c + NF * i : i;
    const int k = kt < m ? kt : m - 1;
    const float live = kt < m ? 1.f : 0.f;
    float2 v[P];
    const float* wk = w + (int64_t)k * L;
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const float ww = live * wk[t + T * e];
      v[e] = make_float2(ww * ua[e], ww * ub[e]);
    }
    fft_wg<L, P, false>(v, my, twl, t);
    const float2* Hk = H + (int64_t)k * L;
#pragma unroll
    for (int e = 0; e < P; ++e) acc[e] = cfma(acc[e], Hk[t + T * e], v[e]);
  }
  if (split && NF > 1) sum_slots<L, P, NF>(acc, lds, c, t);
  fft_wg<L, P, true>(acc, my, twl, t);
  const float sc = 1.0f / (float)L;
  if (keep) {
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int n = t + T * e;
      if (va) y[sa * L + n] = acc[e].x * sc;
      if (vb) y[sb * L + n] = acc[e].y * sc;
    }
  }
}

// x = H_m^* v for signal pairs.
template <int L>
__global__ __launch_bounds__(ffts_per_block(L) * fft_threads(L)) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_adj1d_small(
    const float* __restrict__ vin, float* __restrict__ x, int64_t batch, int m, const float* __restrict__ w,
    const float2* __restrict__ H, const float2* __restrict__ tw, int split) {
  constexpr int P = points_per_thread(L), T = L / P, NF = ffts_per_block(L);
  __shared__ float2 lds[NF * lds_len<L>()];
  __shared__ float2 twl[L];
  stage_twiddles<L>(twl, tw);
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  // split: every slot transforms the pair's input, then takes its terms in turn
  const int64_t pair = split ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * NF + c;
  const int64_t sa = 2 * pair, sb = sa + 1;
  const bool keep = !split || c == 0;
  const bool va = sa < batch, vb = sb < batch;
  float2 V[P];
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int n = t + T * e;
    V[e] = make_float2(va ? vin[sa * L + n] : 0.f, vb ? vin[sb * L + n] : 0.f);
  }
  float2* my = lds + c * lds_len<L>();
  fft_wg<L, P, false>(V, my, twl, t);
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  const int nk = split ? (m + NF - 1) / NF : m;  // same count in every slot (see the forward)
  for (int i = 0; i < nk; ++i) {
    const int kt = split ? c + NF * i : i;
    const int k = kt < m ? kt : m - 1;
    const float live = kt < m ? 1.f : 0.f;
    const float2* Hk = H + (int64_t)k * L;
    float2 g[P];
#pragma unroll
    for (int e = 0; e < P; ++e) g[e] = cmulc(V[e], Hk[t + T * e]);
    fft_wg<L, P, true>(g, my, twl, t);
    const float* wk = w + (int64_t)k * L;
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const float ww = live * wk[t + T * e];
      acc[e].x = fmaf(ww, g[e].x, acc[e].x);
      acc[e].y = fmaf(ww, g[e].y, acc[e].y);
    }
  }
  if (split && NF > 1) sum_slots<L, P, NF>(acc, lds, c, t);
  const float sc = 1.0f / (float)L;
  if (keep) {
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int n = t + T * e;
      if (va) x[sa * L + n] = acc[e].x * sc;
      if (vb) x[sb * L + n] = acc[e].y * sc;
    }
  }
}

template <int L>
static LaunchStatus spec1d_full_t(const float* h, float2* H, int m, const float2* tw, hipStream_t s) {
  constexpr int NF = ffts_per_block(L), T = fft_threads(L);
  const int blocks = (m + NF - 1) / NF;
  hipLaunchKernelGGL(k_spec1d_full<L>, dim3(blocks), dim3(NF * T), 0, s, h, H, m, tw);
  return hipGetLastError();
}

// split the terms over a workgroup's slots when one pair per slot leaves
// compute units idle
static inline bool split_small(int64_t pairs, int NF) { return NF > 1 && (pairs + NF - 1) / NF < 256; }

template <int L>
static LaunchStatus fwd1d_small_t(const Small1D& p, const float* u, float* y, int64_t batch, hipStream_t s,
                                  Tracer* tr) {
  constexpr int NF = ffts_per_block(L), T = fft_threads(L);
  const int64_t pairs = (batch + 1) / 2;
  const bool split = split_small(pairs, NF);
  const int64_t blocks = split ? pairs : (pairs + NF - 1) / NF;
  TraceScope ts(tr, "fwd1d_small", s);
  hipLaunchKernelGGL(k_fwd1d_small<L>, dim3((unsigned)blocks), dim3(NF * T), 0, s, u, y, batch, p.m, p.w, p.H,
                     p.tw, split ? 1 : 0);
  return hipGetLastError();
}

template <int L>
static LaunchStatus adj1d_small_t(const Small1D& p, const float* v, float* x, int64_t batch, hipStream_t s,
                                  Tracer* tr) {
  constexpr int NF = ffts_per_block(L), T = fft_threads(L);
  const int64_t pairs = (batch + 1) / 2;
  const bool split = split_small(pairs, NF);
  const int64_t blocks = split ? pairs : (pairs + NF - 1) / NF;
  TraceScope ts(tr, "adj1d_small", s);
  hipLaunchKernelGGL(k_adj1d_small<L>, dim3((unsigned)blocks), dim3(NF * T), 0, s, v, x, batch, p.m, p.w, p.H,
                     p.tw, split ? 1 : 0);
  return hipGetLastError();
}

LaunchStatus launch_spec1d_full(int L, const float* h, float2* H, int m, const float2* tw, hipStream_t s) {
  switch (L) {
#define PC_CASE(LL) \
  case LL:          \
    return spec1d_full_t<LL>(h, H, m, tw, s);
    PC_FOR_EACH_L(PC_CASE)
#undef PC_CASE
  }
  return hipErrorInvalidValue;
}

LaunchStatus launch_fwd1d_small(const Small1D& p, const float* u, float* y, int64_t batch, hipStream_t s,
                                Tracer* tr) {
  switch (p.L) {
#define PC_CASE(LL) \
  case LL:          \
    return fwd1d_small_t<LL>(p, u, y, batch, s, tr);
    PC_FOR_EACH_L(PC_CASE)
#undef PC_CASE
  }
  return hipErrorInvalidValue;
}

LaunchStatus launch_adj1d_small(const Small1D& p, const float* v, float* x, int64_t batch, hipStream_t s,
                                Tracer* tr) {
  switch (p.L) {
#define PC_CASE(LL) \
  case LL:          \
    return adj1d_small_t<LL>(p, v, x, batch, s, tr);
    PC_FOR_EACH_L(PC_CASE)
#undef PC_CASE
  }
  return hipErrorInvalidValue;
}

// ===========================================================================
// N = R * L: four-step split n = n2 + L n1, f = f1 + R f2
//
//   X[f1 + R f2] = FFT_L(a^{f1})[f2],
//   a^{f1}[n2]   = W_N^{f1 n2} sum_{n1} x[n2 + L n1] W_R^{f1 n1},
//
// with W_M = exp(-2 i pi / M).  The inverse runs the same split backwards:
//   y[n2 + L n1] = (1/N) sum_{f1} W_R^{-f1 n1} W_N^{-f1 n2} b^{f1}[n2],
//   b^{f1} = unnormalised inverse FFT_L of the class-f1 spectrum.
//
// A windowed term z = w_k . u with support [o, o + S) is transformed from its
// own origin: with z'[d] = z[o + d],
//   Z[f] = W_N^{f o} sum_d z'[d] W_N^{f d},
// so the fold reads the support contiguously (d = slot index) and the phase
// W_N^{f o} is carried by the stored spectra, Hd[k][f1][f2] =
// H_k[f] W_N^{f o_k} with f = f1 + R f2.  The adjoint uses the same frame:
// conj(Hd_k) already carries the phase W_N^{-f o_k} that restricting the
// inverse transform to the window needs.
// W_N^{f1 d} comes from the class table twC[f1 * L + d] (coalesced in d);
// W_R^{j} = twN[j * L].
// ===========================================================================

// LDS pad period of the four-step kernels' exchanges
constexpr int FPAD = 32;

// LDS exchange buffers of the four-step transform kernels.  Workgroups of 512
// or more threads use two, with ping-pong exchanges (at the register counts of
// these kernels such a workgroup is alone on its compute unit, so the second
// buffer costs no occupancy); smaller workgroups use one.
template <int L, int P>
constexpr bool fs_pingpong() {
  return L / P >= 512 || 2 * lds_len<L, FPAD>() * 8 <= 80 * 1024;
}
template <int L, int P>
constexpr int fs_lds_len() {
  return (fs_pingpong<L, P>() ? 2 : 1) * lds_len<L, FPAD>();
}
template <int L, int P>
struct FsLds {
  float2* buf[2];
  __device__ explicit FsLds(float2* lds) : buf{lds, fs_pingpong<L, P>() ? lds + lds_len<L, FPAD>() : lds} {}
  // one transform with the thread's register twiddles
  template <bool INV, int NT>
  __device__ __forceinline__ void fft(float2 (&v)[P], const float2 (&twr)[NT], int t) {
    if constexpr (fs_pingpong<L, P>()) {
      fft_wg_reg_pp<L, P, INV, FPAD>(v, buf, twr, t);
      if constexpr (fft_exchanges<L, P>() % 2 == 1) {
        float2* x = buf[0];
        buf[0] = buf[1];
        buf[1] = x;
      }
    } else {
      fft_wg_reg<L, P, INV, FPAD>(v, buf[0], twr, t);
    }
  }
};

template <int L, int R>
__device__ __forceinline__ float2 unit_root_R(const float2* __restrict__ twN, int j) {
  return twN[(j % R) * L];
}

// Load base[i] through a 32-bit unsigned byte offset from a uniform base, so
// that the address is one SGPR pair plus one VGPR (no 64-bit arithmetic).
template <class X>
__device__ __forceinline__ X ldu(const X* __restrict__ base, uint32_t i) {
  return *reinterpret_cast<const X*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(X));
}

// Every L-long block that the four-step kernels pass between launches (class
// spectra Hd and Vws, class outputs Bws, gradient partials E, the modulated
// windows cw) keeps element f2 = t + T e at block_pos(f2, T) (T = L / P):
// the thread that holds f2 in the workgroup transform moves elements e and
// e + 1 with one 16-byte access, and a wave's access covers 1 KiB
// contiguously.
template <int L, int P>
__device__ __forceinline__ int block_elem(int j) {  // inverse of block_pos
  constexpr int T = L / P;
  const int blk = j / (2 * T), r = j % (2 * T);
  return (r >> 1) + T * (2 * blk + (r & 1));
}

template <int L, int P>
__device__ __forceinline__ void load_blk(const float2* __restrict__ b, float2 (&v)[P], int t) {
  static_assert(P % 2 == 0, "even points per thread");
  constexpr int T = L / P;
  const float4* b4 = reinterpret_cast<const float4*>(b);
#pragma unroll
  for (int h = 0; h < P / 2; ++h) {
    const float4 q = ldu(b4, (uint32_t)(h * T + t));
    v[2 * h] = make_float2(q.x, q.y);
    v[2 * h + 1] = make_float2(q.z, q.w);
  }
}

template <int L, int P>
__device__ __forceinline__ void store_blk(float2* __restrict__ b, const float2 (&v)[P], int t) {
  constexpr int T = L / P;
  float4* b4 = reinterpret_cast<float4*>(b);
#pragma unroll
  for (int h = 0; h < P / 2; ++h)
    b4[h * T + t] = make_float4(v[2 * h].x, v[2 * h].y, v[2 * h + 1].x, v[2 * h + 1].y);
}

// (o + d) mod N for o < N, d < N
template <uint32_t N>
__device__ __forceinline__ uint32_t wrapN(uint32_t n) {
  if constexpr ((N & (N - 1)) == 0)
    return n & (N - 1);
  else
    return min(n, n - N);  // n - N wraps above n when n < N
}

// a^{f1}[d] = sum_{c < C} cw_k^{f1,c}[d] z[o + c L + d] with
// cw_k^{f1,c}[d] = w_k[o + c L + d] W_N^{f1 (c L + d)}, for a windowed term
// whose support [o, o + S) is at most C L long (cw is zero beyond S; C is 1
// or 2, and C L <= N).  The chunk c of cw starts at cwb + c L.  All loads are
// issued before any is used.
template <int L, int R, int P, int C>
__device__ __forceinline__ void fold_short(float2 (&v)[P], int t, const float* __restrict__ xa,
                                           const float* __restrict__ xb, int o,
                                           const float2* __restrict__ cwb) {
  static_assert(C == 1 || C == 2, "one or two chunks");
  constexpr int T = L / P;
  constexpr uint32_t N = (uint32_t)L * R;
  float ra[C][P], rb[C][P];
  float2 rc[C][P];
#pragma unroll
  for (int c = 0; c < C; ++c) {
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const uint32_t n = wrapN<N>((uint32_t)o + (uint32_t)(c * L + t + T * e));  // o < N, c L + d < N
      ra[c][e] = ldu(xa, n);
      rb[c][e] = ldu(xb, n);
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c) load_blk<L, P>(cwb + c * L, rc[c], t);
#pragma unroll
  for (int e = 0; e < P; ++e) {
    float2 a = cmul(make_float2(ra[0][e], rb[0][e]), rc[0][e]);
#pragma unroll
    for (int c = 1; c < C; ++c) a = cfma(a, make_float2(ra[c][e], rb[c][e]), rc[c][e]);
    v[e] = a;
  }
}

// Same for supports longer than L: a^{f1}[d] = W_N^{f1 d} sum_c z[o + d + c L] W_R^{f1 c}.
template <int L, int R, int P>
__device__ __forceinline__ void fold_long(float2 (&v)[P], int t, int f1, const float* __restrict__ xa,
                                          const float* __restrict__ xb, const float* __restrict__ wc,
                                          int o, int S, const float2* __restrict__ twC,
                                          const float2* __restrict__ twN) {
  constexpr int T = L / P;
  constexpr uint32_t N = (uint32_t)L * R;
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int d0 = t + T * e;
    float2 a = make_float2(0.f, 0.f);
    int c = 0;
    for (int d = d0; d < S; d += L, ++c) {
      const uint32_t n = wrapN<N>((uint32_t)(o + d));
      const float ww = ldu(wc, (uint32_t)d);
      const float2 z = make_float2(ww * ldu(xa, n), ww * ldu(xb, n));
      a = cfma(a, z, unit_root_R<L, R>(twN, f1 * c));
    }
    v[e] = cmul(a, ldu(twC, (uint32_t)(f1 * L + d0)));
  }
}

// Class spectra of whole signals: out[(sig*R + f1)*L + f2] = X_sig[f1 + R f2].
// pairs = true packs signals (2i, 2i+1) as one complex signal.
template <int L, int R, int P>
__global__ __launch_bounds__(L / P) void k_fold_fft(const float* __restrict__ x, int64_t n_sig, bool pairs,
                                                             float2* __restrict__ out, const float2* __restrict__ tw,
                                                             const float2* __restrict__ twC,
                                                             const float2* __restrict__ twN,
                                                             const float* __restrict__ zeros) {
  constexpr int T = L / P, N = L * R;
  // one transform per workgroup: the twiddles are read from the (cached)
  // global table rather than staged, which also leaves room for two
  // workgroups per CU
  __shared__ float2 lds[lds_len<L, FPAD>()];
  const int t = threadIdx.x;
  // the R class workgroups of a signal (pair) each read the whole signal:
  // numbered so that they run on one XCD and the signal is fetched once
  const int64_t b = xcd_major(blockIdx.x, gridDim.x);
  const int f1 = (int)(b % R);
  const int64_t idx = b / R;
  // the imaginary part: the pair's second signal, or N zeros (no pair)
  const float* xa;
  const float* xb = zeros;
  if (pairs) {
    xa = x + 2 * idx * N;
    if (2 * idx + 1 < n_sig) xb = xa + N;
  } else {
    xa = x + idx * N;
  }
  float2 wr[R];
#pragma unroll
  for (int n1 = 0; n1 < R; ++n1) wr[n1] = unit_root_R<L, R>(twN, f1 * n1);
  const float2* tc = twC + f1 * L;
  float2 v[P];
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int n2 = t + T * e;
    float2 a = make_float2(0.f, 0.f);
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) {
      const float2 z = make_float2(xa[n2 + L * n1], xb[n2 + L * n1]);
      a = cfma(a, z, wr[n1]);
    }
    v[e] = cmul(a, tc[n2]);
  }
  fft_wg<L, P, false, FPAD>(v, lds, tw, t);
  store_blk<L, P>(out + (idx * R + f1) * L, v, t);
}

// Forward, class f1 of one signal pair: sum_k Hd_k^{f1} . FFT_L(fold(w_k u)),
// then the class's inverse FFT_L, stored for the combine step.
// C: chunks of the short-support path (1 or 2; the plan's cw table), 0 for
// the long-support path.
template <int L, int R, int P, int C>
__global__ __launch_bounds__(L / P) void k_fwd1d_large(const float* __restrict__ u, int64_t batch, Large1D p) {
  constexpr int N = L * R;
  __shared__ float2 lds[fs_lds_len<L, P>()];
  FsLds<L, P> xl(lds);
  const int t = threadIdx.x;
  // the thread's twiddles stay in registers for all m + 1 transforms
  float2 twr[tw_reg_count<L, P>()];
  load_tw_reg<L, P>(twr, p.tw, t);
  const int f1 = blockIdx.x % R;
  const int64_t pair = blockIdx.x / R;
  const float* xa = u + 2 * pair * N;
  const float* xb = 2 * pair + 1 < batch ? xa + N : p.zeros;  // odd batch: a zero second signal
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  for (int k = 0; k < p.m; ++k) {
    const int S = p.w_len[k];
    if (S == 0) continue;
    const int o = p.w_off[k];
    const float* wc = p.wc + p.w_base[k];
    (void)wc;
    float2 v[P];
    if constexpr (C > 0)
      fold_short<L, R, P, C>(v, t, xa, xb, o, p.cw + ((int64_t)k * R + f1) * C * L);
    else
      fold_long<L, R, P>(v, t, f1, xa, xb, wc, o, S, p.twC, p.twN);
    // the spectrum loads are issued before the transform so that their
    // latency overlaps it
    float2 hv[P];
    load_blk<L, P>(p.Hd + ((int64_t)k * R + f1) * L, hv, t);
    xl.template fft<false>(v, twr, t);
#pragma unroll
    for (int e = 0; e < P; ++e) acc[e] = cfma(acc[e], hv[e], v[e]);
  }
  xl.template fft<true>(acc, twr, t);
  store_blk<L, P>(p.Bws + (pair * R + f1) * L, acc, t);
}

// y[n2 + L n1] = (1/N) sum_f1 W_R^{-f1 n1} (W_N^{-f1 n2} b^{f1}[n2]).
// One thread per 16-byte pair of a block (block_pos: elements n2 = t + T e
// and n2 + T, e even), so every class block is read with coalesced 16-byte
// loads.
template <int L, int R, int P>
__global__ __launch_bounds__(256) void k_combine1d(const float2* __restrict__ Bws, float* __restrict__ y, int64_t batch,
                                                   const float2* __restrict__ twC) {
  constexpr int N = L * R, T = L / P;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pairs = (batch + 1) / 2;
  if (gid >= pairs * (L / 2)) return;
  const int64_t pair = gid / (L / 2);
  const int q = (int)(gid % (L / 2));  // float4 index inside a block: h T + t
  const int h = q / T, t = q % T;
  const int n2[2] = {t + T * 2 * h, t + T * (2 * h + 1)};
  float2 b[2][R];
#pragma unroll
  for (int f1 = 0; f1 < R; ++f1) {
    const float4 v = reinterpret_cast<const float4*>(Bws + (pair * R + f1) * L)[q];
    b[0][f1] = cmulc(make_float2(v.x, v.y), twC[f1 * L + n2[0]]);
    b[1][f1] = cmulc(make_float2(v.z, v.w), twC[f1 * L + n2[1]]);
  }
  const float sc = 1.0f / (float)N;
  const int64_t sa = 2 * pair, sb = sa + 1;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    dftR<R, true>(b[j]);
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) y[sa * N + n2[j] + L * n1] = b[j][n1].x * sc;
    if (sb < batch) {
#pragma unroll
      for (int n1 = 0; n1 < R; ++n1) y[sb * N + n2[j] + L * n1] = b[j][n1].y * sc;
    }
  }
}

// Adjoint, one item of one signal pair: g = F(conj(H_k) . V) on the item's
// samples, assembled class by class, times the window; stored for the
// overlap-add.  Long-support plans (C = 0) have one item per chunk of at most
// L samples of a term's support.  Short-support plans (C = 1 or 2) have one
// item per term, whose support is at most C L long: the R class transforms
// serve all its chunks, and each chunk takes its window and class modulation
// together from cw.
template <int L, int R, int P, int C>
__global__ __launch_bounds__(L / P) void k_adj1d_large(Large1D p) {
  constexpr int T = L / P;
  __shared__ float2 lds[fs_lds_len<L, P>()];
  FsLds<L, P> xl(lds);
  const int t = threadIdx.x;
  // the thread's twiddles stay in registers for all R transforms
  float2 twr[tw_reg_count<L, P>()];
  load_tw_reg<L, P>(twr, p.tw, t);
  const int item = blockIdx.x % p.n_items;
  const int64_t pair = blockIdx.x / p.n_items;
  const int k = p.item_k[item];
  const int c0 = p.item_d0[item];
  const int Sc = p.item_len[item];
  const int chunk = c0 / L;  // long path: chunks start at multiples of L inside the support
  constexpr int NC = C > 0 ? C : 1;  // accumulators (chunks) per item
  float2 acc[NC][P];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int e = 0; e < P; ++e) acc[c][e] = make_float2(0.f, 0.f);
  const float2* Hk = p.Hd + (int64_t)k * R * L;
  const float2* Vp = p.Vws + pair * R * L;
  auto load = [&](float2(&vv)[P], float2(&hh)[P], int f1) {
    load_blk<L, P>(Vp + f1 * L, vv, t);
    load_blk<L, P>(Hk + f1 * L, hh, t);
  };
  auto prod = [&](float2(&vv)[P], const float2(&hh)[P]) {
#pragma unroll
    for (int e = 0; e < P; ++e) vv[e] = cmulc(vv[e], hh[e]);
  };
  // class f1: inverse FFT_L of conj(Hd) . V, back-modulated by W_N^{-f1 d}
  // (chunks after the first also carry W_R^{-f1 chunk}) and summed
  auto step = [&](float2(&vv)[P], int f1) {
    xl.template fft<true>(vv, twr, t);
    if constexpr (C > 0) {
      // chunk c: conj(cw_k^{f1,c}) carries W_N^{-f1 (c L + d)} and the window
#pragma unroll
      for (int c = 0; c < C; ++c) {
        float2 rt[P];
        load_blk<L, P>(p.cw + (((int64_t)k * R + f1) * C + c) * L, rt, t);
        // slots at or beyond Sc accumulate values that are never stored
#pragma unroll
        for (int e = 0; e < P; ++e) acc[c][e] = cfma_conj(acc[c][e], rt[e], vv[e]);  // + vv conj(rt), 4 FMAs
      }
    } else {
      float2 rt[P];
      const float2* tc = p.twC + f1 * L;
#pragma unroll
      for (int e = 0; e < P; ++e) rt[e] = ldu(tc, (uint32_t)(t + T * e));
      if (chunk != 0) {
        const float2 u = unit_root_R<L, R>(p.twN, f1 * chunk);
#pragma unroll
        for (int e = 0; e < P; ++e) rt[e] = cmul(rt[e], u);
      }
#pragma unroll
      for (int e = 0; e < P; ++e) acc[0][e] = cfma_conj(acc[0][e], rt[e], vv[e]);
    }
  };
  // (prefetching the next class into a second register set measured slower
  // than register-resident twiddles, which need those registers)
  for (int f1 = 0; f1 < R; ++f1) {
    float2 va[P], ha[P];
    load(va, ha, f1);
    prod(va, ha);
    step(va, f1);
  }
  float2* out = p.Pws + pair * p.p_stride + p.item_out[item];
  const float sc = 1.0f / (float)(L * R);
  if constexpr (C > 0) {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < P; ++e) {
        const int d = c * L + t + T * e;
        if (d < Sc) out[d] = cscale(acc[c][e], sc);
      }
  } else {
    const float* wc = p.wc + p.w_base[k] + c0;
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int d = t + T * e;
      if (d < Sc) out[d] = cscale(acc[0][e], wc[d] * sc);
    }
  }
}

// x[n] = sum over the items covering n of their stored products; the items
// that can cover a sample are listed per tile of 256 samples.
template <int L, int R>
__global__ __launch_bounds__(256) void k_ola1d(Large1D p, float* __restrict__ x, int64_t batch) {
  constexpr int N = L * R, TILES = N / 256;
  // one workgroup per (pair, tile): the tile's item list is uniform
  const int64_t pair = blockIdx.x / TILES;
  const int tile = (int)(blockIdx.x % TILES);
  const int n = tile * 256 + (int)threadIdx.x;
  const float2* base = p.Pws + pair * p.p_stride;
  float2 acc = make_float2(0.f, 0.f);
  const int j0 = p.tile_off[tile], j1 = p.tile_off[tile + 1];
  for (int j = j0; j < j1; ++j) {
    const int it = p.tile_items[j];
    int dd = n - p.item_oc[it];
    if (dd < 0) dd += N;
    if (dd < p.item_len[it]) acc = cadd(acc, base[p.item_out[it] + dd]);
  }
  const int64_t sa = 2 * pair, sb = sa + 1;
  x[sa * N + n] = acc.x;
  if (sb < batch) x[sb * N + n] = acc.y;
}

// (L, R, P) instantiations of the four-step kernels; P (points per thread)
// is a plan-time choice.
#define PC_FOR_EACH_LRP(X)                                                          \
  X(8192, 2, 16) X(8192, 4, 16) X(8192, 8, 16) X(8192, 16, 16)                     \
  X(6144, 2, 24) X(6144, 4, 24) X(6144, 8, 24) X(6144, 16, 24)                     \
  X(4096, 2, 16) X(4096, 4, 16) X(4096, 8, 16) X(4096, 16, 16)

bool fourstep_variant_supported(int L, int R, int P) {
#define PC_CASE(LL, RR, PP) \
  if (L == LL && R == RR && P == PP) return true;
  PC_FOR_EACH_LRP(PC_CASE)
#undef PC_CASE
  return false;
}

template <int L, int R, int P>
static LaunchStatus fold_fft_t(const Large1D& p, const float* x, int64_t n_sig, float2* out, bool pairs,
                               hipStream_t s, Tracer* tr) {
  const int64_t nb = pairs ? (n_sig + 1) / 2 : n_sig;
  TraceScope ts(tr, "fold_fft", s);
  hipLaunchKernelGGL((k_fold_fft<L, R, P>), dim3((unsigned)(nb * R)), dim3(L / P), 0, s, x, n_sig, pairs, out, p.tw,
                     p.twC, p.twN, p.zeros);
  return hipGetLastError();
}

template <int L, int R, int P>
static LaunchStatus fwd1d_large_t(const Large1D& p, const float* u, float* y, int64_t batch, hipStream_t s,
                                  Tracer* tr) {
  const int64_t pairs = (batch + 1) / 2;
  {
    TraceScope ts(tr, "fwd1d_large", s);
    const dim3 grid((unsigned)(pairs * R)), block(L / P);
    if (p.chunks == 2)
      hipLaunchKernelGGL((k_fwd1d_large<L, R, P, 2>), grid, block, 0, s, u, batch, p);
    else if (p.chunks == 1)
      hipLaunchKernelGGL((k_fwd1d_large<L, R, P, 1>), grid, block, 0, s, u, batch, p);
    else
      hipLaunchKernelGGL((k_fwd1d_large<L, R, P, 0>), grid, block, 0, s, u, batch, p);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nthr = pairs * (L / 2);
  TraceScope ts(tr, "combine1d", s);
  hipLaunchKernelGGL((k_combine1d<L, R, P>), dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, p.Bws, y, batch,
                     p.twC);
  return hipGetLastError();
}

template <int L, int R, int P>
static LaunchStatus adj1d_large_t(const Large1D& p, const float* v, float* x, int64_t batch, hipStream_t s,
                                  Tracer* tr) {
  const int64_t pairs = (batch + 1) / 2;
  LaunchStatus e = fold_fft_t<L, R, P>(p, v, batch, p.Vws, true, s, tr);
  if (e != hipSuccess) return e;
  if (p.n_items > 0) {
    TraceScope ts(tr, "adj1d_large", s);
    const dim3 grid((unsigned)(pairs * p.n_items)), block(L / P);
    if (p.chunks == 2)
      hipLaunchKernelGGL((k_adj1d_large<L, R, P, 2>), grid, block, 0, s, p);
    else if (p.chunks == 1)
      hipLaunchKernelGGL((k_adj1d_large<L, R, P, 1>), grid, block, 0, s, p);
    else
      hipLaunchKernelGGL((k_adj1d_large<L, R, P, 0>), grid, block, 0, s, p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  TraceScope ts(tr, "ola1d", s);
  hipLaunchKernelGGL((k_ola1d<L, R>), dim3((unsigned)(pairs * (L * R / 256))), dim3(256), 0, s, p, x, batch);
  return hipGetLastError();
}

LaunchStatus launch_fold_fft(const Large1D& p, const float* x, int64_t n_sig, float2* out, bool pairs,
                             hipStream_t s, Tracer* tr) {
#define PC_CASE(LL, RR, PP) \
  if (p.L == LL && p.R == RR && p.P == PP) return fold_fft_t<LL, RR, PP>(p, x, n_sig, out, pairs, s, tr);
  PC_FOR_EACH_LRP(PC_CASE)
#undef PC_CASE
  return hipErrorInvalidValue;
}

LaunchStatus launch_fwd1d_large(const Large1D& p, const float* u, float* y, int64_t batch, hipStream_t s,
                                Tracer* tr) {
#define PC_CASE(LL, RR, PP) \
  if (p.L == LL && p.R == RR && p.P == PP) return fwd1d_large_t<LL, RR, PP>(p, u, y, batch, s, tr);
  PC_FOR_EACH_LRP(PC_CASE)
#undef PC_CASE
  return hipErrorInvalidValue;
}

LaunchStatus launch_adj1d_large(const Large1D& p, const float* v, float* x, int64_t batch, hipStream_t s,
                                Tracer* tr) {
#define PC_CASE(LL, RR, PP) \
  if (p.L == LL && p.R == RR && p.P == PP) return adj1d_large_t<LL, RR, PP>(p, v, x, batch, s, tr);
  PC_FOR_EACH_LRP(PC_CASE)
#undef PC_CASE
  return hipErrorInvalidValue;
}

// ===========================================================================
// Spectra as parameters: import / export in the natural half-spectrum layout
// spec[k][f], f <= N/2 (the layout of a real FFT), and the gradient of a
// scalar loss with respect to them.
//
// The internal spectra are full and Hermitian (they multiply pair-packed
// complex signals), so an imported half-spectrum is extended by conjugate
// symmetry with the imaginary parts at DC and Nyquist dropped, the values an
// inverse real transform ignores.
//
// Gradient: with Z = F^*(w_k . u) and Gh = F^*(dL/dy) for a real signal, the
// gradient with respect to spec[k][f] (convention dL/dRe + i dL/dIm) is
// (c_f / N) conj(Z[f]) Gh[f], c_f = 1 at DC and Nyquist, 2 elsewhere.  For a
// pair-packed signal with full spectra A = F^*(w_k . (u_a + i u_b)) and
// C = F^*(g_a + i g_b), the sum over the two signals of conj(Z[f]) Gh[f] is
// (E[f] + conj(E[-f])) / 2 with E = conj(A) . C, so the kernels accumulate E
// over pairs and combine f with -f at the end.
// ===========================================================================

__device__ __forceinline__ float half_weight(int f, int n) { return (f == 0 || 2 * f == n) ? 1.f : 2.f; }

__device__ __forceinline__ float2 hermitian_value(const float2* __restrict__ half, int f, int n) {
  if (2 * f <= n) {
    float2 v = half[f];
    if (f == 0 || 2 * f == n) v.y = 0.f;
    return v;
  }
  return cconj(half[n - f]);
}

template <int L>
__global__ __launch_bounds__(256) void k_import1d_small(const float2* __restrict__ spec, float2* __restrict__ H, int m) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)m * L) return;
  const int k = (int)(gid / L), f = (int)(gid % L);
  H[gid] = hermitian_value(spec + (int64_t)k * (L / 2 + 1), f, L);
}

template <int L>
__global__ __launch_bounds__(256) void k_export1d_small(const float2* __restrict__ H, float2* __restrict__ spec,
                                                        int m) {
  constexpr int NH = L / 2 + 1;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)m * NH) return;
  const int k = (int)(gid / NH), f = (int)(gid % NH);
  spec[gid] = H[(int64_t)k * L + f];
}

// Full spectra of pair-packed signals: out[pair][f] = F^*(x_a + i x_b)[f].
template <int L>
__global__ __launch_bounds__(ffts_per_block(L) * fft_threads(L)) void k_fft_pairs_small(
    const float* __restrict__ x, int64_t batch, float2* __restrict__ out, const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(L), T = L / P, NF = ffts_per_block(L);
  __shared__ float2 lds[NF * lds_len<L>()];
  __shared__ float2 twl[L];
  stage_twiddles<L>(twl, tw);
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int64_t pair = (int64_t)blockIdx.x * NF + c;
  const int64_t sa = 2 * pair, sb = sa + 1;
  const bool va = sa < batch, vb = sb < batch;
  float2 v[P];
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int n = t + T * e;
    v[e] = make_float2(va ? x[sa * L + n] : 0.f, vb ? x[sb * L + n] : 0.f);
  }
  fft_wg<L, P, false>(v, lds + c * lds_len<L>(), twl, t);
  if (va) {
#pragma unroll
    for (int e = 0; e < P; ++e) out[pair * L + t + T * e] = v[e];
  }
}

// gspec[k][f] for f <= N/2, one term per FFT slot, looping over the pairs.
template <int L>
__global__ __launch_bounds__(ffts_per_block(L) * fft_threads(L)) void k_grad1d_small(
    const float* __restrict__ u, int64_t batch, int m, const float* __restrict__ w, const float2* __restrict__ Gc,
    float2* __restrict__ gspec, const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(L), T = L / P, NF = ffts_per_block(L), NH = L / 2 + 1;
  __shared__ float2 lds[NF * lds_len<L>()];
  __shared__ float2 twl[L];
  stage_twiddles<L>(twl, tw);
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int kraw = blockIdx.x * NF + c;
  const bool ok = kraw < m;
  const int k = ok ? kraw : m - 1;
  float2* my = lds + c * lds_len<L>();
  const float* wk = w + (int64_t)k * L;
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  const int64_t pairs = (batch + 1) / 2;
  for (int64_t pr = 0; pr < pairs; ++pr) {
    const int64_t sa = 2 * pr, sb = sa + 1;
    const bool vb = sb < batch;
    float2 v[P];
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int n = t + T * e;
      const float ww = wk[n];
      v[e] = make_float2(ww * u[sa * L + n], vb ? ww * u[sb * L + n] : 0.f);
    }
    fft_wg<L, P, false>(v, my, twl, t);
#pragma unroll
    for (int e = 0; e < P; ++e) acc[e] = cfma_conj(acc[e], v[e], Gc[pr * L + t + T * e]);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < P; ++e) my[lpad(t + T * e)] = acc[e];
  __syncthreads();
  if (ok) {
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int f = t + T * e;
      if (f < NH) {
        const float2 a = my[lpad(f)];
        const float2 b = my[lpad(f == 0 ? 0 : L - f)];
        const float sc = 0.5f * half_weight(f, L) / (float)L;
        gspec[(int64_t)k * NH + f] = make_float2(sc * (a.x + b.x), sc * (a.y - b.y));
      }
    }
  }
}

// ---- four-step layout -------------------------------------------------------

// The four-step path stores its spectra in the frame of each window's origin
// o_k: Hd[k][f1][f2] = H_k[f] W_N^{f o_k}, f = f1 + R f2.
template <int L, int R>
__device__ __forceinline__ float2 origin_phase(const float2* __restrict__ twN, int f, int o) {
  constexpr int N = L * R;
  return twN[(int)(((int64_t)f * o) % N)];
}

template <int L, int R, int P>
__global__ __launch_bounds__(256) void k_import1d_large(const float2* __restrict__ spec, float2* __restrict__ Hd,
                                                        int m, const int* __restrict__ w_off,
                                                        const float2* __restrict__ twN) {
  constexpr int N = L * R;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)m * N) return;
  const int k = (int)(gid / N);
  const int rem = (int)(gid % N);
  const int f = rem / L + R * block_elem<L, P>(rem % L);
  Hd[gid] = cmul(hermitian_value(spec + (int64_t)k * (N / 2 + 1), f, N), origin_phase<L, R>(twN, f, w_off[k]));
}

template <int L, int R, int P>
__global__ __launch_bounds__(256) void k_export1d_large(const float2* __restrict__ Hd, float2* __restrict__ spec,
                                                        int m, const int* __restrict__ w_off,
                                                        const float2* __restrict__ twN) {
  constexpr int N = L * R, NH = N / 2 + 1;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)m * NH) return;
  const int k = (int)(gid / NH), f = (int)(gid % NH);
  spec[gid] =
      cmulc(Hd[((int64_t)k * R + f % R) * L + block_pos(f / R, L / P)], origin_phase<L, R>(twN, f, w_off[k]));
}

// In place: natural-frame spectra (from the whole-signal transform of h_k)
// to the window-origin frame.
template <int L, int R, int P>
__global__ __launch_bounds__(256) void k_origin_phase1d(float2* __restrict__ Hd, int m, const int* __restrict__ w_off,
                                                        const float2* __restrict__ twN) {
  constexpr int N = L * R;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)m * N) return;
  const int k = (int)(gid / N);
  const int rem = (int)(gid % N);
  const int f = rem / L + R * block_elem<L, P>(rem % L);
  Hd[gid] = cmul(Hd[gid], origin_phase<L, R>(twN, f, w_off[k]));
}

// E_k^{f1} = sum over pairs of conj(FFT_L(fold(w_k u))) . Gdec^{f1}, one
// (term, class) per workgroup.
template <int L, int R, int P, int C>
__global__ __launch_bounds__(L / P) void k_grad1d_large(const float* __restrict__ u, int64_t batch, Large1D p,
                                                        float2* __restrict__ E) {
  constexpr int N = L * R;
  __shared__ float2 lds[fs_lds_len<L, P>()];
  FsLds<L, P> xl(lds);
  const int t = threadIdx.x;
  float2 twr[tw_reg_count<L, P>()];
  load_tw_reg<L, P>(twr, p.tw, t);
  const int f1 = blockIdx.x % R;
  const int k = blockIdx.x / R;
  const int S = p.w_len[k];
  const int o = p.w_off[k];
  const float* wc = p.wc + p.w_base[k];
  (void)wc;
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  const int64_t pairs = (batch + 1) / 2;
  if (S > 0) {
    for (int64_t pr = 0; pr < pairs; ++pr) {
      const float* xa = u + 2 * pr * N;
      const float* xb = 2 * pr + 1 < batch ? xa + N : p.zeros;
      float2 v[P];
      if constexpr (C > 0)
        fold_short<L, R, P, C>(v, t, xa, xb, o, p.cw + ((int64_t)k * R + f1) * C * L);
      else
        fold_long<L, R, P>(v, t, f1, xa, xb, wc, o, S, p.twC, p.twN);
      float2 gv[P];
      load_blk<L, P>(p.Vws + (pr * R + f1) * L, gv, t);
      xl.template fft<false>(v, twr, t);
#pragma unroll
      for (int e = 0; e < P; ++e) acc[e] = cfma_conj(acc[e], v[e], gv[e]);
    }
  }
  store_blk<L, P>(E + ((int64_t)k * R + f1) * L, acc, t);
}

template <int L, int R, int P>
__global__ __launch_bounds__(256) void k_grad_export1d_large(const float2* __restrict__ E, float2* __restrict__ gspec,
                                                             int m, const int* __restrict__ w_off,
                                                             const float2* __restrict__ twN) {
  constexpr int N = L * R, NH = N / 2 + 1;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)m * NH) return;
  const int k = (int)(gid / NH), f = (int)(gid % NH);
  const int fm = (N - f) % N;
  // E was accumulated with the windowed transforms in the window-origin
  // frame; the natural-frame product carries conj(W_N^{f o_k})
  constexpr int T = L / P;
  const float2 a =
      cmulc(E[((int64_t)k * R + f % R) * L + block_pos(f / R, T)], origin_phase<L, R>(twN, f, w_off[k]));
  const float2 b =
      cmulc(E[((int64_t)k * R + fm % R) * L + block_pos(fm / R, T)], origin_phase<L, R>(twN, fm, w_off[k]));
  const float sc = 0.5f * half_weight(f, N) / (float)N;
  gspec[gid] = make_float2(sc * (a.x + b.x), sc * (a.y - b.y));
}

// out[i] = conj(in[i]); in may equal out
__global__ __launch_bounds__(256) void k_conj(const float2* in, float2* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = cconj(in[i]);
}

// ---- launchers --------------------------------------------------------------

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

LaunchStatus launch_conj(const float2* in, float2* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_conj, dim3(blocks_for(n)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

LaunchStatus launch_spectra1d(const Small1D* ps, const Large1D* pl, const float2* in, float2* out, bool import,
                              hipStream_t s) {
  if (ps) {
    const Small1D& p = *ps;
    switch (p.L) {
#define PC_CASE(LL)                                                                                              \
  case LL:                                                                                                       \
    if (import)                                                                                                  \
      hipLaunchKernelGGL(k_import1d_small<LL>, dim3(blocks_for((int64_t)p.m * LL)), dim3(256), 0, s, in,         \
                         const_cast<float2*>(p.H), p.m);                                                         \
    else                                                                                                         \
      hipLaunchKernelGGL(k_export1d_small<LL>, dim3(blocks_for((int64_t)p.m * (LL / 2 + 1))), dim3(256), 0, s,   \
                         p.H, out, p.m);                                                                         \
    return hipGetLastError();
      PC_FOR_EACH_L(PC_CASE)
#undef PC_CASE
    }
    return hipErrorInvalidValue;
  }
  const Large1D& p = *pl;
#define PC_CASE(LL, RR, PP)                                                                                     \
  if (p.L == LL && p.R == RR && p.P == PP) {                                                                    \
    if (import)                                                                                                 \
      hipLaunchKernelGGL((k_import1d_large<LL, RR, PP>), dim3(blocks_for((int64_t)p.m * LL * RR)), dim3(256), 0, \
                         s, in, const_cast<float2*>(p.Hd), p.m, p.w_off, p.twN);                                \
    else                                                                                                        \
      hipLaunchKernelGGL((k_export1d_large<LL, RR, PP>), dim3(blocks_for((int64_t)p.m * (LL * RR / 2 + 1))),    \
                         dim3(256), 0, s, p.Hd, out, p.m, p.w_off, p.twN);                                      \
    return hipGetLastError();                                                                                   \
  }
  PC_FOR_EACH_LRP(PC_CASE)
#undef PC_CASE
  return hipErrorInvalidValue;
}

LaunchStatus launch_origin_phase1d(const Large1D& p, float2* Hd, hipStream_t s) {
#define PC_CASE(LL, RR, PP)                                                                                  \
  if (p.L == LL && p.R == RR && p.P == PP) {                                                                 \
    hipLaunchKernelGGL((k_origin_phase1d<LL, RR, PP>), dim3(blocks_for((int64_t)p.m * LL * RR)), dim3(256), 0, \
                       s, Hd, p.m, p.w_off, p.twN);                                                          \
    return hipGetLastError();                                                                                \
  }
  PC_FOR_EACH_LRP(PC_CASE)
#undef PC_CASE
  return hipErrorInvalidValue;
}

template <int L>
static LaunchStatus grad1d_small_t(const Small1D& p, const float* u, const float* gy, float2* gspec, int64_t batch,
                                   float2* work, hipStream_t s) {
  constexpr int NF = ffts_per_block(L), T = fft_threads(L);
  const int64_t pairs = (batch + 1) / 2;
  hipLaunchKernelGGL(k_fft_pairs_small<L>, dim3((unsigned)((pairs + NF - 1) / NF)), dim3(NF * T), 0, s, gy, batch,
                     work, p.tw);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad1d_small<L>, dim3((unsigned)((p.m + NF - 1) / NF)), dim3(NF * T), 0, s, u, batch, p.m,
                     p.w, work, gspec, p.tw);
  return hipGetLastError();
}

LaunchStatus launch_grad1d_small(const Small1D& p, const float* u, const float* gy, float2* gspec, int64_t batch,
                                 float2* work, hipStream_t s, Tracer* tr) {
  TraceScope ts(tr, "grad1d_small", s);
  switch (p.L) {
#define PC_CASE(LL) \
  case LL:          \
    return grad1d_small_t<LL>(p, u, gy, gspec, batch, work, s);
    PC_FOR_EACH_L(PC_CASE)
#undef PC_CASE
  }
  return hipErrorInvalidValue;
}

template <int L, int R, int P>
static LaunchStatus grad1d_large_t(const Large1D& p, const float* u, const float* gy, float2* gspec, int64_t batch,
                                   float2* E, hipStream_t s, Tracer* tr) {
  LaunchStatus e = fold_fft_t<L, R, P>(p, gy, batch, p.Vws, true, s, tr);
  if (e != hipSuccess) return e;
  {
    TraceScope ts(tr, "grad1d_large", s);
    const dim3 grid((unsigned)(p.m * R)), block(L / P);
    if (p.chunks == 2)
      hipLaunchKernelGGL((k_grad1d_large<L, R, P, 2>), grid, block, 0, s, u, batch, p, E);
    else if (p.chunks == 1)
      hipLaunchKernelGGL((k_grad1d_large<L, R, P, 1>), grid, block, 0, s, u, batch, p, E);
    else
      hipLaunchKernelGGL((k_grad1d_large<L, R, P, 0>), grid, block, 0, s, u, batch, p, E);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_grad_export1d_large<L, R, P>), dim3(blocks_for((int64_t)p.m * (L * R / 2 + 1))), dim3(256), 0,
                     s, E, gspec, p.m, p.w_off, p.twN);
  return hipGetLastError();
}

LaunchStatus launch_grad1d_large(const Large1D& p, const float* u, const float* gy, float2* gspec, int64_t batch,
                                 float2* E, hipStream_t s, Tracer* tr) {
#define PC_CASE(LL, RR, PP) \
  if (p.L == LL && p.R == RR && p.P == PP) return grad1d_large_t<LL, RR, PP>(p, u, gy, gspec, batch, E, s, tr);
  PC_FOR_EACH_LRP(PC_CASE)
#undef PC_CASE
  return hipErrorInvalidValue;
}

}  // namespace pc
