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

// Plan-time spectra H_k = F^* h_k (full complex, natural order).
template <int L>
__global__ __launch_bounds__(ffts_per_block(L) * fft_threads(L)) void k_spec1d_full(
    const float* __restrict__ h, float2* __restrict__ H, int m, const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(L), T = L / P, NF = ffts_per_block(L);
  __shared__ float2 lds[NF * lds_len<L>()];
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int k = blockIdx.x * NF + c;
  const bool ok = k < m;
  float2 v[P];
#pragma unroll
  for (int e = 0; e < P; ++e) v[e] = make_float2(ok ? h[(int64_t)k * L + t + T * e] : 0.f, 0.f);
  fft_wg<L, P, false>(v, lds + c * lds_len<L>(), tw, t);
  if (ok) {
#pragma unroll
    for (int e = 0; e < P; ++e) H[(int64_t)k * L + t + T * e] = v[e];
  }
}

// y = H_m u for signal pairs.
template <int L>
__global__ __launch_bounds__(ffts_per_block(L) * fft_threads(L)) void k_fwd1d_small(
    const float* __restrict__ u, float* __restrict__ y, int64_t batch, int m, const float* __restrict__ w,
    const float2* __restrict__ H, const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(L), T = L / P, NF = ffts_per_block(L);
  __shared__ float2 lds[NF * lds_len<L>()];
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int64_t pair = (int64_t)blockIdx.x * NF + c;
  const int64_t sa = 2 * pair, sb = sa + 1;
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
  for (int k = 0; k < m; ++k) {
    float2 v[P];
    const float* wk = w + (int64_t)k * L;
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const float ww = wk[t + T * e];
      v[e] = make_float2(ww * ua[e], ww * ub[e]);
    }
    fft_wg<L, P, false>(v, my, tw, t);
    const float2* Hk = H + (int64_t)k * L;
#pragma unroll
    for (int e = 0; e < P; ++e) acc[e] = cfma(acc[e], Hk[t + T * e], v[e]);
  }
  fft_wg<L, P, true>(acc, my, tw, t);
  const float sc = 1.0f / (float)L;
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int n = t + T * e;
    if (va) y[sa * L + n] = acc[e].x * sc;
    if (vb) y[sb * L + n] = acc[e].y * sc;
  }
}

// x = H_m^* v for signal pairs.
template <int L>
__global__ __launch_bounds__(ffts_per_block(L) * fft_threads(L)) void k_adj1d_small(
    const float* __restrict__ vin, float* __restrict__ x, int64_t batch, int m, const float* __restrict__ w,
    const float2* __restrict__ H, const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(L), T = L / P, NF = ffts_per_block(L);
  __shared__ float2 lds[NF * lds_len<L>()];
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int64_t pair = (int64_t)blockIdx.x * NF + c;
  const int64_t sa = 2 * pair, sb = sa + 1;
  const bool va = sa < batch, vb = sb < batch;
  float2 V[P];
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int n = t + T * e;
    V[e] = make_float2(va ? vin[sa * L + n] : 0.f, vb ? vin[sb * L + n] : 0.f);
  }
  float2* my = lds + c * lds_len<L>();
  fft_wg<L, P, false>(V, my, tw, t);
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  for (int k = 0; k < m; ++k) {
    const float2* Hk = H + (int64_t)k * L;
    float2 g[P];
#pragma unroll
    for (int e = 0; e < P; ++e) g[e] = cmulc(V[e], Hk[t + T * e]);
    fft_wg<L, P, true>(g, my, tw, t);
    const float* wk = w + (int64_t)k * L;
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const float ww = wk[t + T * e];
      acc[e].x = fmaf(ww, g[e].x, acc[e].x);
      acc[e].y = fmaf(ww, g[e].y, acc[e].y);
    }
  }
  const float sc = 1.0f / (float)L;
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int n = t + T * e;
    if (va) x[sa * L + n] = acc[e].x * sc;
    if (vb) x[sb * L + n] = acc[e].y * sc;
  }
}

template <int L>
static LaunchStatus spec1d_full_t(const float* h, float2* H, int m, const float2* tw, hipStream_t s) {
  constexpr int NF = ffts_per_block(L), T = fft_threads(L);
  const int blocks = (m + NF - 1) / NF;
  hipLaunchKernelGGL(k_spec1d_full<L>, dim3(blocks), dim3(NF * T), 0, s, h, H, m, tw);
  return hipGetLastError();
}

template <int L>
static LaunchStatus fwd1d_small_t(const Small1D& p, const float* u, float* y, int64_t batch, hipStream_t s,
                                  Tracer* tr) {
  constexpr int NF = ffts_per_block(L), T = fft_threads(L);
  const int64_t pairs = (batch + 1) / 2;
  const int64_t blocks = (pairs + NF - 1) / NF;
  TraceScope ts(tr, "fwd1d_small", s);
  hipLaunchKernelGGL(k_fwd1d_small<L>, dim3((unsigned)blocks), dim3(NF * T), 0, s, u, y, batch, p.m, p.w, p.H,
                     p.tw);
  return hipGetLastError();
}

template <int L>
static LaunchStatus adj1d_small_t(const Small1D& p, const float* v, float* x, int64_t batch, hipStream_t s,
                                  Tracer* tr) {
  constexpr int NF = ffts_per_block(L), T = fft_threads(L);
  const int64_t pairs = (batch + 1) / 2;
  const int64_t blocks = (pairs + NF - 1) / NF;
  TraceScope ts(tr, "adj1d_small", s);
  hipLaunchKernelGGL(k_adj1d_small<L>, dim3((unsigned)blocks), dim3(NF * T), 0, s, v, x, batch, p.m, p.w, p.H,
                     p.tw);
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
//   a^{f1}[n2]   = sum_{n1} x[n2 + L n1] exp(-2 i pi f1 (n2 + L n1) / N).
//
// A window of compact support folds into a^{f1} from its support only.  The
// inverse runs the same split backwards:
//   y[n2 + L n1] = (1/N) sum_{f1} exp(+2 i pi f1 (n2 + L n1)/N) b^{f1}[n2],
//   b^{f1} = unnormalised inverse FFT_L of the class-f1 spectrum.
// ===========================================================================

// a^{f1}[n2] over the support [o, o + S) (mod N) of a (window x signal)
// product.  wc = null means a window equal to one on the support.
template <int L, int R>
__device__ __forceinline__ float2 fold_one(int n2, int f1, const float* __restrict__ xa, const float* __restrict__ xb,
                                           const float* __restrict__ wc, int o, int S,
                                           const float2* __restrict__ twN) {
  constexpr int N = L * R;
  int d = n2 - (o % L);
  if (d < 0) d += L;
  float2 a = make_float2(0.f, 0.f);
  for (; d < S; d += L) {
    int n = o + d;
    if (n >= N) n -= N;
    const float ww = wc ? wc[d] : 1.0f;
    const float2 z = make_float2(ww * xa[n], xb ? ww * xb[n] : 0.f);
    const unsigned ti = ((unsigned)f1 * (unsigned)n) % (unsigned)N;
    a = cfma(a, z, twN[ti]);
  }
  return a;
}

// Class spectra of whole signals: out[(sig*R + f1)*L + f2] = X_sig[f1 + R f2].
// pairs = true packs signals (2i, 2i+1) as one complex signal.
template <int L, int R>
__global__ __launch_bounds__(fft_threads(L)) void k_fold_fft(const float* __restrict__ x, int64_t n_sig, bool pairs,
                                                             float2* __restrict__ out, const float2* __restrict__ tw,
                                                             const float2* __restrict__ twN) {
  constexpr int P = points_per_thread(L), T = L / P, N = L * R;
  __shared__ float2 lds[lds_len<L>()];
  const int t = threadIdx.x;
  const int f1 = blockIdx.x % R;
  const int64_t idx = blockIdx.x / R;
  const float* xa;
  const float* xb = nullptr;
  if (pairs) {
    xa = x + 2 * idx * N;
    if (2 * idx + 1 < n_sig) xb = xa + N;
  } else {
    xa = x + idx * N;
  }
  float2 v[P];
#pragma unroll
  for (int e = 0; e < P; ++e) v[e] = fold_one<L, R>(t + T * e, f1, xa, xb, nullptr, 0, N, twN);
  fft_wg<L, P, false>(v, lds, tw, t);
  float2* o = out + (idx * R + f1) * L;
#pragma unroll
  for (int e = 0; e < P; ++e) o[t + T * e] = v[e];
}

// Forward, class f1 of one signal pair: sum_k Hd_k^{f1} . FFT_L(fold(w_k u)),
// then the class's inverse FFT_L, stored for the combine step.
template <int L, int R>
__global__ __launch_bounds__(fft_threads(L)) void k_fwd1d_large(const float* __restrict__ u, int64_t batch,
                                                                Large1D p) {
  constexpr int P = points_per_thread(L), T = L / P, N = L * R;
  __shared__ float2 lds[lds_len<L>()];
  const int t = threadIdx.x;
  const int f1 = blockIdx.x % R;
  const int64_t pair = blockIdx.x / R;
  const float* xa = u + 2 * pair * N;
  const float* xb = (2 * pair + 1 < batch) ? xa + N : nullptr;
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  for (int k = 0; k < p.m; ++k) {
    const int S = p.w_len[k];
    if (S == 0) continue;
    const int o = p.w_off[k];
    const float* wc = p.wc + p.w_base[k];
    float2 v[P];
#pragma unroll
    for (int e = 0; e < P; ++e) v[e] = fold_one<L, R>(t + T * e, f1, xa, xb, wc, o, S, p.twN);
    fft_wg<L, P, false>(v, lds, p.tw, t);
    const float2* Hk = p.Hd + ((int64_t)k * R + f1) * L;
#pragma unroll
    for (int e = 0; e < P; ++e) acc[e] = cfma(acc[e], Hk[t + T * e], v[e]);
  }
  fft_wg<L, P, true>(acc, lds, p.tw, t);
  float2* o = p.Bws + (pair * R + f1) * L;
#pragma unroll
  for (int e = 0; e < P; ++e) o[t + T * e] = acc[e];
}

// y[n2 + L n1] = (1/N) sum_f1 W_R^{-f1 n1} (W_N^{-f1 n2} b^{f1}[n2]).
template <int L, int R>
__global__ __launch_bounds__(256) void k_combine1d(const float2* __restrict__ Bws, float* __restrict__ y, int64_t batch,
                                                   const float2* __restrict__ twN) {
  constexpr int N = L * R;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pairs = (batch + 1) / 2;
  if (gid >= pairs * L) return;
  const int64_t pair = gid / L;
  const int n2 = (int)(gid % L);
  float2 b[R];
#pragma unroll
  for (int f1 = 0; f1 < R; ++f1) b[f1] = cmulc(Bws[(pair * R + f1) * L + n2], twN[f1 * n2]);
  dftR<R, true>(b);
  const float sc = 1.0f / (float)N;
  const int64_t sa = 2 * pair, sb = sa + 1;
#pragma unroll
  for (int n1 = 0; n1 < R; ++n1) y[sa * N + n2 + L * n1] = b[n1].x * sc;
  if (sb < batch) {
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) y[sb * N + n2 + L * n1] = b[n1].y * sc;
  }
}

// Adjoint, one (term, support chunk) item of one signal pair:
// g = F(conj(H_k) . V) restricted to the chunk, assembled class by class,
// then multiplied by the window and stored for the overlap-add.
template <int L, int R>
__global__ __launch_bounds__(fft_threads(L)) void k_adj1d_large(Large1D p) {
  constexpr int P = points_per_thread(L), T = L / P, N = L * R;
  __shared__ float2 lds[lds_len<L>()];
  const int t = threadIdx.x;
  const int item = blockIdx.x % p.n_items;
  const int64_t pair = blockIdx.x / p.n_items;
  const int k = p.item_k[item];
  const int c0 = p.item_d0[item];
  const int S = p.w_len[k];
  const int Sc = (S - c0) < L ? (S - c0) : L;
  int oc = p.w_off[k] + c0;
  if (oc >= N) oc -= N;
  const int ocL = oc % L;
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  for (int f1 = 0; f1 < R; ++f1) {
    const float2* Hk = p.Hd + ((int64_t)k * R + f1) * L;
    const float2* Vp = p.Vws + (pair * R + f1) * L;
    float2 g[P];
#pragma unroll
    for (int e = 0; e < P; ++e) g[e] = cmulc(Vp[t + T * e], Hk[t + T * e]);
    fft_wg<L, P, true>(g, lds, p.tw, t);
#pragma unroll
    for (int e = 0; e < P; ++e) {
      int dd = t + T * e - ocL;
      if (dd < 0) dd += L;
      if (dd < Sc) {
        int n = oc + dd;
        if (n >= N) n -= N;
        const unsigned ti = ((unsigned)f1 * (unsigned)n) % (unsigned)N;
        acc[e] = cfma(acc[e], g[e], cconj(p.twN[ti]));
      }
    }
  }
  const float* wc = p.wc + p.w_base[k] + c0;
  float2* out = p.Pws + pair * p.p_stride + p.item_out[item];
  const float sc = 1.0f / (float)N;
#pragma unroll
  for (int e = 0; e < P; ++e) {
    int dd = t + T * e - ocL;
    if (dd < 0) dd += L;
    if (dd < Sc) out[dd] = cscale(acc[e], wc[dd] * sc);
  }
}

// x[n] = sum over items covering n of their stored products.
template <int L, int R>
__global__ __launch_bounds__(256) void k_ola1d(Large1D p, float* __restrict__ x, int64_t batch) {
  constexpr int N = L * R;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pairs = (batch + 1) / 2;
  if (gid >= pairs * N) return;
  const int64_t pair = gid / N;
  const int n = (int)(gid % N);
  const float2* base = p.Pws + pair * p.p_stride;
  float2 acc = make_float2(0.f, 0.f);
  for (int it = 0; it < p.n_items; ++it) {
    const int k = p.item_k[it];
    const int c0 = p.item_d0[it];
    const int S = p.w_len[k];
    const int Sc = (S - c0) < L ? (S - c0) : L;
    int oc = p.w_off[k] + c0;
    if (oc >= N) oc -= N;
    int dd = n - oc;
    if (dd < 0) dd += N;
    if (dd < Sc) acc = cadd(acc, base[p.item_out[it] + dd]);
  }
  const int64_t sa = 2 * pair, sb = sa + 1;
  x[sa * N + n] = acc.x;
  if (sb < batch) x[sb * N + n] = acc.y;
}

#define PC_FOR_EACH_LR(X)                                               \
  X(8192, 2) X(8192, 4) X(8192, 8) X(8192, 16) X(6144, 2) X(6144, 4) \
  X(6144, 8) X(6144, 16)

template <int L, int R>
static LaunchStatus fold_fft_t(const Large1D& p, const float* x, int64_t n_sig, float2* out, bool pairs,
                               hipStream_t s, Tracer* tr) {
  const int64_t nb = pairs ? (n_sig + 1) / 2 : n_sig;
  TraceScope ts(tr, "fold_fft", s);
  hipLaunchKernelGGL((k_fold_fft<L, R>), dim3((unsigned)(nb * R)), dim3(fft_threads(L)), 0, s, x, n_sig, pairs, out,
                     p.tw, p.twN);
  return hipGetLastError();
}

template <int L, int R>
static LaunchStatus fwd1d_large_t(const Large1D& p, const float* u, float* y, int64_t batch, hipStream_t s,
                                  Tracer* tr) {
  const int64_t pairs = (batch + 1) / 2;
  {
    TraceScope ts(tr, "fwd1d_large", s);
    hipLaunchKernelGGL((k_fwd1d_large<L, R>), dim3((unsigned)(pairs * R)), dim3(fft_threads(L)), 0, s, u, batch, p);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nthr = pairs * L;
  TraceScope ts(tr, "combine1d", s);
  hipLaunchKernelGGL((k_combine1d<L, R>), dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, p.Bws, y, batch,
                     p.twN);
  return hipGetLastError();
}

template <int L, int R>
static LaunchStatus adj1d_large_t(const Large1D& p, const float* v, float* x, int64_t batch, hipStream_t s,
                                  Tracer* tr) {
  const int64_t pairs = (batch + 1) / 2;
  LaunchStatus e = fold_fft_t<L, R>(p, v, batch, p.Vws, true, s, tr);
  if (e != hipSuccess) return e;
  if (p.n_items > 0) {
    TraceScope ts(tr, "adj1d_large", s);
    hipLaunchKernelGGL((k_adj1d_large<L, R>), dim3((unsigned)(pairs * p.n_items)), dim3(fft_threads(L)), 0, s, p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t nthr = pairs * (int64_t)L * R;
  TraceScope ts(tr, "ola1d", s);
  hipLaunchKernelGGL((k_ola1d<L, R>), dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, p, x, batch);
  return hipGetLastError();
}

LaunchStatus launch_fold_fft(const Large1D& p, const float* x, int64_t n_sig, float2* out, bool pairs,
                             hipStream_t s, Tracer* tr) {
#define PC_CASE(LL, RR) \
  if (p.L == LL && p.R == RR) return fold_fft_t<LL, RR>(p, x, n_sig, out, pairs, s, tr);
  PC_FOR_EACH_LR(PC_CASE)
#undef PC_CASE
  return hipErrorInvalidValue;
}

LaunchStatus launch_fwd1d_large(const Large1D& p, const float* u, float* y, int64_t batch, hipStream_t s,
                                Tracer* tr) {
#define PC_CASE(LL, RR) \
  if (p.L == LL && p.R == RR) return fwd1d_large_t<LL, RR>(p, u, y, batch, s, tr);
  PC_FOR_EACH_LR(PC_CASE)
#undef PC_CASE
  return hipErrorInvalidValue;
}

LaunchStatus launch_adj1d_large(const Large1D& p, const float* v, float* x, int64_t batch, hipStream_t s,
                                Tracer* tr) {
#define PC_CASE(LL, RR) \
  if (p.L == LL && p.R == RR) return adj1d_large_t<LL, RR>(p, v, x, batch, s, tr);
  PC_FOR_EACH_LR(PC_CASE)
#undef PC_CASE
  return hipErrorInvalidValue;
}

}  // namespace pc
