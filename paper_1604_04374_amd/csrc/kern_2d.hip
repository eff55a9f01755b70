// 2D kernels of the convolution-product expansion on an N1 x N2 periodic
// image (row-major, N2 contiguous); the higher-dimensional extension of
// section 5.2 with index pairs taken modulo (N1, N2).
//
// The 2D transform is taken as real row transforms followed by complex
// column transforms on the N2/2 + 1 retained column frequencies (the
// half-spectrum of a real image).  Two real rows are packed into one complex
// row transform and separated with the conjugate symmetry of real data.
//
// Spectral planes (row-transformed images, spectra, partial sums) are stored
// column-major: plane[f2][n1], so every column transform reads and writes
// one contiguous vector.  The row kernels work on tiles of 2G rows and
// transpose through LDS, so that their spectral-plane accesses are runs of
// 2G consecutive entries.
//
// Forward:  rows:  RA_q = rowFFT(b_q . u)                       (q = column factor)
//           cols:  S_g = sum_{k in group g} H_k . colFFT(a_k1 . RA_k2)
//                  T = colIFFT(sum_g S_g)
//           rows:  y = rowIFFT(T) / (N1 N2)
// Adjoint:  rows:  V = rowFFT(v);  cols: V <- colFFT(V)
//           cols:  Q_q = sum_k1 a_k1 . colIFFT(conj(H_k) . V)   (one slot per (column, q))
//           rows:  x = sum_q b_q . rowIFFT(Q_q) / (N1 N2)
// With dense (non-separable) windows q runs over the m terms, a = 1 and
// b_q = w_q.
#include "fft_engine.hpp"
#include "pc_internal.hpp"

namespace pc {

#define PC_FOR_EACH_L2(X) \
  X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192) \
  X(96) X(192) X(384) X(768) X(1536) X(3072) X(6144)

// Window applied by the row kernels.
enum RowWin { RW_NONE = 0, RW_FACTOR = 1, RW_DENSE = 2 };

__device__ __forceinline__ void row_weights(const float* __restrict__ wsrc, int mode, int q, int N1, int L2, int r,
                                            int n2, float& wa, float& wb) {
  if (mode == RW_FACTOR) {
    wa = wb = wsrc[(int64_t)q * L2 + n2];
  } else if (mode == RW_DENSE) {
    const float* base = wsrc + ((int64_t)q * N1 + r) * L2 + n2;
    wa = base[0];
    wb = base[L2];
  } else {
    wa = wb = 1.0f;
  }
}

// ---------------------------------------------------------------------------
// row kernels: G row pairs (2G rows) per workgroup
// ---------------------------------------------------------------------------

// Row pairs per workgroup: as many as LDS allows (transform buffers plus the
// twiddle table within 156 KiB), at most 8 (tiles of 16 rows).
constexpr int row_pairs_per_block(int L2) {
  int g = 8;
  while (g > 1 && (g * (L2 + L2 / 16) + L2) * 8 > 156 * 1024) g /= 2;
  return g;
}

// Half-spectra of windowed rows, transposed: out[q][img][f2][n1], f2 < H2.
template <int L2>
__global__ __launch_bounds__(row_pairs_per_block(L2) * fft_threads(L2)) void k_rows_fwd(
    const float* __restrict__ x, int N1, const float* __restrict__ wsrc, int mode, float2* __restrict__ out,
    int64_t q_stride, const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(L2), T = L2 / P, G = row_pairs_per_block(L2), H2 = L2 / 2 + 1;
  constexpr int NT = G * T;
  __shared__ float2 lds[G * lds_len<L2>()];
  __shared__ float2 twl[L2];
  stage_twiddles<L2>(twl, tw);
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int blocks_per_img = N1 / (2 * G);
  const int64_t img = blockIdx.x / blocks_per_img;
  const int r0 = (blockIdx.x % blocks_per_img) * 2 * G;
  const int r = r0 + 2 * c;
  const int q = blockIdx.y;
  const float* ra = x + (img * N1 + r) * L2;
  float2 v[P];
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int n2 = t + T * e;
    float wa, wb;
    row_weights(wsrc, mode, q, N1, L2, r, n2, wa, wb);
    v[e] = make_float2(wa * ra[n2], wb * ra[n2 + L2]);
  }
  float2* my = lds + c * lds_len<L2>();
  fft_wg<L2, P, false>(v, my, twl, t);
  __syncthreads();
#pragma unroll
  for (int e = 0; e < P; ++e) my[lpad(t + T * e)] = v[e];
  __syncthreads();
  // separate the two rows: U_a = (C[f] + conj C[-f]) / 2, U_b = (C[f] - conj C[-f]) / (2 i)
  float2 ua[P], ub[P];
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int f = t + T * e;
    const float2 cf = my[lpad(f)];
    const float2 cm = my[lpad(f == 0 ? 0 : L2 - f)];
    ua[e] = make_float2(0.5f * (cf.x + cm.x), 0.5f * (cf.y - cm.y));
    ub[e] = make_float2(0.5f * (cf.y + cm.y), -0.5f * (cf.x - cm.x));
  }
  __syncthreads();
  // transpose through LDS: tile[f][row in block]
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int f = t + T * e;
    if (f < H2) {
      lds[f * (2 * G) + 2 * c] = ua[e];
      lds[f * (2 * G) + 2 * c + 1] = ub[e];
    }
  }
  __syncthreads();
  float2* o = out + (int64_t)q * q_stride + img * ((int64_t)H2 * N1) + r0;
  for (int idx = threadIdx.x; idx < H2 * 2 * G; idx += NT) {
    const int f = idx / (2 * G), ri = idx % (2 * G);
    o[(int64_t)f * N1 + ri] = lds[idx];
  }
}

// Real rows from transposed half-spectra:
// out[img][n1][n2] = scale * sum_q w_q . rowIFFT(in[q][img][:, n1]).
template <int L2>
__global__ __launch_bounds__(row_pairs_per_block(L2) * fft_threads(L2)) void k_rows_inv(
    const float2* __restrict__ in, int nq, int64_t q_stride, int N1, const float* __restrict__ wsrc, int mode,
    float* __restrict__ out, float scale, const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(L2), T = L2 / P, G = row_pairs_per_block(L2), H2 = L2 / 2 + 1;
  constexpr int NT = G * T;
  __shared__ float2 lds[G * lds_len<L2>()];
  __shared__ float2 twl[L2];
  stage_twiddles<L2>(twl, tw);
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int blocks_per_img = N1 / (2 * G);
  const int64_t img = blockIdx.x / blocks_per_img;
  const int r0 = (blockIdx.x % blocks_per_img) * 2 * G;
  const int r = r0 + 2 * c;
  float2* my = lds + c * lds_len<L2>();
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  for (int q = 0; q < nq; ++q) {
    const float2* src = in + (int64_t)q * q_stride + img * ((int64_t)H2 * N1) + r0;
    __syncthreads();  // the previous transform is done with LDS
    for (int idx = threadIdx.x; idx < H2 * 2 * G; idx += NT) {
      const int f = idx / (2 * G), ri = idx % (2 * G);
      lds[idx] = src[(int64_t)f * N1 + ri];
    }
    __syncthreads();
    float2 v[P];
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int f = t + T * e;
      float2 a, b;
      if (f < H2) {
        a = lds[f * (2 * G) + 2 * c];
        b = lds[f * (2 * G) + 2 * c + 1];
        if (f == 0 || f == L2 / 2) {  // the inverse real transform ignores these imaginary parts
          a.y = 0.f;
          b.y = 0.f;
        }
      } else {
        a = cconj(lds[(L2 - f) * (2 * G) + 2 * c]);
        b = cconj(lds[(L2 - f) * (2 * G) + 2 * c + 1]);
      }
      v[e] = make_float2(a.x - b.y, a.y + b.x);  // a + i b
    }
    fft_wg<L2, P, true>(v, my, twl, t);
#pragma unroll
    for (int e = 0; e < P; ++e) {
      float wa, wb;
      row_weights(wsrc, mode, q, N1, L2, r, t + T * e, wa, wb);
      acc[e].x = fmaf(wa, v[e].x, acc[e].x);
      acc[e].y = fmaf(wb, v[e].y, acc[e].y);
    }
  }
  float* oa = out + (img * N1 + r) * L2;
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int n2 = t + T * e;
    oa[n2] = acc[e].x * scale;
    oa[n2 + L2] = acc[e].y * scale;
  }
}

// ---------------------------------------------------------------------------
// column kernels: NF columns per workgroup, each column contiguous
// ---------------------------------------------------------------------------

// Forward column pass for the term group blockIdx.y: the group takes the
// column factors q in [q0, q1) and, for each, every row factor k1 (the
// column of RA_q is loaded once and reused for all of them).
// ngroups == 1: T = colIFFT(S) is written directly; otherwise the partial
// spectrum S_g goes to part[g] for the summing kernel.
template <int L1>
__global__ __launch_bounds__(ffts_per_block(L1) * fft_threads(L1)) void k_cols_fwd(
    const float2* __restrict__ RA, int64_t q_stride, int H2, int m1, int m2, int dense,
    const float* __restrict__ wrows, const float2* __restrict__ Hs, int ngroups, float2* __restrict__ Tout,
    float2* __restrict__ part, int64_t part_stride, const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(L1), T = L1 / P, NF = ffts_per_block(L1);
  __shared__ float2 lds[NF * lds_len<L1>()];
  __shared__ float2 twl[L1];
  stage_twiddles<L1>(twl, tw);
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int nblk = (H2 + NF - 1) / NF;
  const int64_t img = blockIdx.x / nblk;
  const int f2raw = (blockIdx.x % nblk) * NF + c;
  const bool valid = f2raw < H2;
  const int f2 = valid ? f2raw : H2 - 1;  // idle slots recompute a valid column and store nothing
  const int64_t plane = (int64_t)L1 * H2;
  const int nq = dense ? m1 * m2 : m2;  // dense windows: q runs over all terms
  const int g = blockIdx.y;
  const int q0 = (int)((int64_t)nq * g / ngroups), q1 = (int)((int64_t)nq * (g + 1) / ngroups);
  const int nk1 = dense ? 1 : m1;
  float2* my = lds + c * lds_len<L1>();
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  for (int q = q0; q < q1; ++q) {
    const float2* col = RA + q * q_stride + img * plane + (int64_t)f2 * L1;
    float2 cv[P];
#pragma unroll
    for (int e = 0; e < P; ++e) cv[e] = col[t + T * e];
    for (int k1 = 0; k1 < nk1; ++k1) {
      const int k = dense ? q : k1 * m2 + q;
      const float2* Hk = Hs + (int64_t)k * plane + (int64_t)f2 * L1;
      float2 hv[P], v[P];
#pragma unroll
      for (int e = 0; e < P; ++e) hv[e] = Hk[t + T * e];
#pragma unroll
      for (int e = 0; e < P; ++e) v[e] = dense ? cv[e] : cscale(cv[e], wrows[(int64_t)k1 * L1 + t + T * e]);
      fft_wg<L1, P, false>(v, my, twl, t);
#pragma unroll
      for (int e = 0; e < P; ++e) acc[e] = cfma(acc[e], hv[e], v[e]);
    }
  }
  if (ngroups == 1) {
    fft_wg<L1, P, true>(acc, my, twl, t);
    if (valid) {
      float2* dst = Tout + img * plane + (int64_t)f2 * L1;
#pragma unroll
      for (int e = 0; e < P; ++e) dst[t + T * e] = acc[e];
    }
  } else if (valid) {
    float2* dst = part + g * part_stride + img * plane + (int64_t)f2 * L1;
#pragma unroll
    for (int e = 0; e < P; ++e) dst[t + T * e] = acc[e];
  }
}

// T[img][f2][:] = colIFFT(sum_g part[g][img][f2][:]).
template <int L1>
__global__ __launch_bounds__(ffts_per_block(L1) * fft_threads(L1)) void k_cols_sum_inv(
    const float2* __restrict__ part, int64_t part_stride, int ngroups, int H2, float2* __restrict__ Tout,
    const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(L1), T = L1 / P, NF = ffts_per_block(L1);
  __shared__ float2 lds[NF * lds_len<L1>()];
  __shared__ float2 twl[L1];
  stage_twiddles<L1>(twl, tw);
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int nblk = (H2 + NF - 1) / NF;
  const int64_t img = blockIdx.x / nblk;
  const int f2raw = (blockIdx.x % nblk) * NF + c;
  const bool valid = f2raw < H2;
  const int f2 = valid ? f2raw : H2 - 1;
  const int64_t off = img * ((int64_t)L1 * H2) + (int64_t)f2 * L1;
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = part[off + t + T * e];
  for (int g = 1; g < ngroups; ++g) {
#pragma unroll
    for (int e = 0; e < P; ++e) acc[e] = cadd(acc[e], part[g * part_stride + off + t + T * e]);
  }
  fft_wg<L1, P, true>(acc, lds + c * lds_len<L1>(), twl, t);
  if (valid) {
#pragma unroll
    for (int e = 0; e < P; ++e) Tout[off + t + T * e] = acc[e];
  }
}

// Adjoint column pass, one (column, q) per FFT slot:
// Q_q[img][f2][:] = sum_k1 a_k1 . colIFFT(conj(H_k) . Vh[img][f2][:]).
template <int L1>
__global__ __launch_bounds__(ffts_per_block(L1) * fft_threads(L1)) void k_cols_adj(
    const float2* __restrict__ Vh, int H2, int m1, int m2, int dense, const float* __restrict__ wrows,
    const float2* __restrict__ Hs, float2* __restrict__ Q, int64_t q_stride, const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(L1), T = L1 / P, NF = ffts_per_block(L1);
  __shared__ float2 lds[NF * lds_len<L1>()];
  __shared__ float2 twl[L1];
  stage_twiddles<L1>(twl, tw);
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int nblk = (H2 + NF - 1) / NF;
  const int64_t img = blockIdx.x / nblk;
  const int f2raw = (blockIdx.x % nblk) * NF + c;
  const bool valid = f2raw < H2;
  const int f2 = valid ? f2raw : H2 - 1;
  const int q = blockIdx.y;
  const int64_t plane = (int64_t)L1 * H2;
  const int64_t coff = img * plane + (int64_t)f2 * L1;
  float2 vh[P];
#pragma unroll
  for (int e = 0; e < P; ++e) vh[e] = Vh[coff + t + T * e];
  const int nk1 = dense ? 1 : m1;
  float2* my = lds + c * lds_len<L1>();
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  for (int k1 = 0; k1 < nk1; ++k1) {
    const int k = dense ? q : k1 * m2 + q;
    const float2* Hk = Hs + (int64_t)k * plane + (int64_t)f2 * L1;
    float2 g[P];
#pragma unroll
    for (int e = 0; e < P; ++e) g[e] = cmulc(vh[e], Hk[t + T * e]);
    fft_wg<L1, P, true>(g, my, twl, t);
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const float wv = dense ? 1.0f : wrows[(int64_t)k1 * L1 + t + T * e];
      acc[e].x = fmaf(wv, g[e].x, acc[e].x);
      acc[e].y = fmaf(wv, g[e].y, acc[e].y);
    }
  }
  if (valid) {
    float2* dst = Q + q * q_stride + coff;
#pragma unroll
    for (int e = 0; e < P; ++e) dst[t + T * e] = acc[e];
  }
}

// In-place column FFTs: io[img][f2][:] = colFFT(io[img][f2][:]).
template <int L1>
__global__ __launch_bounds__(ffts_per_block(L1) * fft_threads(L1)) void k_cols_fft(float2* __restrict__ io, int H2,
                                                                                 const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(L1), T = L1 / P, NF = ffts_per_block(L1);
  __shared__ float2 lds[NF * lds_len<L1>()];
  __shared__ float2 twl[L1];
  stage_twiddles<L1>(twl, tw);
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int nblk = (H2 + NF - 1) / NF;
  const int64_t img = blockIdx.x / nblk;
  const int f2raw = (blockIdx.x % nblk) * NF + c;
  const bool valid = f2raw < H2;
  const int f2 = valid ? f2raw : H2 - 1;
  const int64_t off = img * ((int64_t)L1 * H2) + (int64_t)f2 * L1;
  float2 v[P];
#pragma unroll
  for (int e = 0; e < P; ++e) v[e] = io[off + t + T * e];
  fft_wg<L1, P, false>(v, lds + c * lds_len<L1>(), twl, t);
  if (valid) {
#pragma unroll
    for (int e = 0; e < P; ++e) io[off + t + T * e] = v[e];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int L2>
static LaunchStatus rows_fwd_t(const float* x, int N1, int64_t n_img, const float* wsrc, int mode, int nq,
                               float2* out, int64_t q_stride, const float2* tw, hipStream_t s) {
  constexpr int G = row_pairs_per_block(L2), T = fft_threads(L2);
  const int64_t blocks = n_img * (N1 / (2 * G));
  hipLaunchKernelGGL(k_rows_fwd<L2>, dim3((unsigned)blocks, (unsigned)nq), dim3(G * T), 0, s, x, N1, wsrc, mode, out,
                     q_stride, tw);
  return hipGetLastError();
}

template <int L2>
static LaunchStatus rows_inv_t(const float2* in, int nq, int64_t q_stride, int N1, int64_t n_img, const float* wsrc,
                               int mode, float* out, float scale, const float2* tw, hipStream_t s) {
  constexpr int G = row_pairs_per_block(L2), T = fft_threads(L2);
  const int64_t blocks = n_img * (N1 / (2 * G));
  hipLaunchKernelGGL(k_rows_inv<L2>, dim3((unsigned)blocks), dim3(G * T), 0, s, in, nq, q_stride, N1, wsrc, mode, out,
                     scale, tw);
  return hipGetLastError();
}

template <int L1>
static LaunchStatus cols_fwd_t(const Plan2D& p, int64_t n_img, int64_t q_stride, hipStream_t s) {
  constexpr int NF = ffts_per_block(L1), T = fft_threads(L1);
  const int nblk = (p.H2 + NF - 1) / NF;
  const int64_t plane = (int64_t)L1 * p.H2;
  const int ng = p.col_groups;
  hipLaunchKernelGGL(k_cols_fwd<L1>, dim3((unsigned)(nblk * n_img), (unsigned)ng), dim3(NF * T), 0, s, p.RA,
                     q_stride, p.H2, p.m1, p.m2, p.dense ? 1 : 0, p.wrows, p.Hs, ng, p.Tws, p.Part, plane * n_img,
                     p.tw1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ng == 1) return e;
  hipLaunchKernelGGL(k_cols_sum_inv<L1>, dim3((unsigned)(nblk * n_img)), dim3(NF * T), 0, s, p.Part, plane * n_img,
                     ng, p.H2, p.Tws, p.tw1);
  return hipGetLastError();
}

template <int L1>
static LaunchStatus cols_adj_t(const Plan2D& p, int64_t n_img, int64_t q_stride, hipStream_t s) {
  constexpr int NF = ffts_per_block(L1), T = fft_threads(L1);
  const int nblk = (p.H2 + NF - 1) / NF;
  const int nq = p.dense ? p.m : p.m2;
  hipLaunchKernelGGL(k_cols_adj<L1>, dim3((unsigned)(nblk * n_img), (unsigned)nq), dim3(NF * T), 0, s, p.Tws, p.H2,
                     p.m1, p.m2, p.dense ? 1 : 0, p.wrows, p.Hs, p.RA, q_stride, p.tw1);
  return hipGetLastError();
}

template <int L1>
static LaunchStatus cols_fft_t(float2* io, int H2, int64_t n_img, const float2* tw, hipStream_t s) {
  constexpr int NF = ffts_per_block(L1), T = fft_threads(L1);
  const int nblk = (H2 + NF - 1) / NF;
  hipLaunchKernelGGL(k_cols_fft<L1>, dim3((unsigned)(nblk * n_img)), dim3(NF * T), 0, s, io, H2, tw);
  return hipGetLastError();
}

static LaunchStatus rows_fwd(int L2, const float* x, int N1, int64_t n_img, const float* wsrc, int mode, int nq,
                             float2* out, int64_t q_stride, const float2* tw, hipStream_t s, Tracer* tr = nullptr) {
  TraceScope ts(tr, "rows_fwd", s);
  switch (L2) {
#define PC_CASE(LL) \
  case LL:          \
    return rows_fwd_t<LL>(x, N1, n_img, wsrc, mode, nq, out, q_stride, tw, s);
    PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
  }
  return hipErrorInvalidValue;
}

static LaunchStatus rows_inv(int L2, const float2* in, int nq, int64_t q_stride, int N1, int64_t n_img,
                             const float* wsrc, int mode, float* out, float scale, const float2* tw, hipStream_t s,
                             Tracer* tr = nullptr) {
  TraceScope ts(tr, "rows_inv", s);
  switch (L2) {
#define PC_CASE(LL) \
  case LL:          \
    return rows_inv_t<LL>(in, nq, q_stride, N1, n_img, wsrc, mode, out, scale, tw, s);
    PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
  }
  return hipErrorInvalidValue;
}

static LaunchStatus cols_fwd(const Plan2D& p, int64_t n_img, int64_t q_stride, hipStream_t s, Tracer* tr) {
  TraceScope ts(tr, "cols_fwd", s);
  switch (p.N1) {
#define PC_CASE(LL) \
  case LL:          \
    return cols_fwd_t<LL>(p, n_img, q_stride, s);
    PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
  }
  return hipErrorInvalidValue;
}

static LaunchStatus cols_adj(const Plan2D& p, int64_t n_img, int64_t q_stride, hipStream_t s, Tracer* tr) {
  TraceScope ts(tr, "cols_adj", s);
  switch (p.N1) {
#define PC_CASE(LL) \
  case LL:          \
    return cols_adj_t<LL>(p, n_img, q_stride, s);
    PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
  }
  return hipErrorInvalidValue;
}

static LaunchStatus cols_fft(int L1, float2* io, int H2, int64_t n_img, const float2* tw, hipStream_t s,
                             Tracer* tr = nullptr) {
  TraceScope ts(tr, "cols_fft", s);
  switch (L1) {
#define PC_CASE(LL) \
  case LL:          \
    return cols_fft_t<LL>(io, H2, n_img, tw, s);
    PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
  }
  return hipErrorInvalidValue;
}

int col_groups_for(int H2, int64_t batch, int nq) {
  // split the forward column pass over groups of column factors until about
  // eight column transforms per compute unit are in flight
  const int64_t cols = (int64_t)H2 * batch;
  const int64_t target = 256 * 8;
  int g = 1;
  while (g < nq && cols * g < target) g *= 2;
  return g < nq ? g : nq;
}

LaunchStatus launch_spec2d(const Plan2D& p, const float* h, float2* Hs, hipStream_t s) {
  const int64_t plane = (int64_t)p.N1 * p.H2;
  LaunchStatus e = rows_fwd(p.N2, h, p.N1, p.m, nullptr, RW_NONE, 1, Hs, plane * p.m, p.tw2, s);
  if (e != hipSuccess) return e;
  return cols_fft(p.N1, Hs, p.H2, p.m, p.tw1, s);
}

LaunchStatus launch_fwd2d(const Plan2D& p, const float* u, float* y, int64_t batch, hipStream_t s, Tracer* tr) {
  const int64_t plane = (int64_t)p.N1 * p.H2;
  const int64_t q_stride = plane * batch;
  const int nq = p.dense ? p.m : p.m2;
  LaunchStatus e = rows_fwd(p.N2, u, p.N1, batch, p.wcols, p.dense ? RW_DENSE : RW_FACTOR, nq, p.RA, q_stride,
                            p.tw2, s, tr);
  if (e != hipSuccess) return e;
  e = cols_fwd(p, batch, q_stride, s, tr);
  if (e != hipSuccess) return e;
  const float scale = 1.0f / ((float)p.N1 * (float)p.N2);
  return rows_inv(p.N2, p.Tws, 1, 0, p.N1, batch, nullptr, RW_NONE, y, scale, p.tw2, s, tr);
}

LaunchStatus launch_adj2d(const Plan2D& p, const float* v, float* x, int64_t batch, hipStream_t s, Tracer* tr) {
  const int64_t plane = (int64_t)p.N1 * p.H2;
  const int64_t q_stride = plane * batch;
  const int nq = p.dense ? p.m : p.m2;
  LaunchStatus e = rows_fwd(p.N2, v, p.N1, batch, nullptr, RW_NONE, 1, p.Tws, q_stride, p.tw2, s, tr);
  if (e != hipSuccess) return e;
  e = cols_fft(p.N1, p.Tws, p.H2, batch, p.tw1, s, tr);
  if (e != hipSuccess) return e;
  e = cols_adj(p, batch, q_stride, s, tr);
  if (e != hipSuccess) return e;
  const float scale = 1.0f / ((float)p.N1 * (float)p.N2);
  return rows_inv(p.N2, p.RA, nq, q_stride, p.N1, batch, p.wcols, p.dense ? RW_DENSE : RW_FACTOR, x, scale, p.tw2,
                  s, tr);
}

// ===========================================================================
// Spectra as parameters (natural layout spec[k][f1][f2], f2 <= N2/2, the
// layout of a real 2D FFT) and the gradient of a scalar loss with respect to
// them: dL/dspec[k][f1][f2] = (c_f2 / N) sum_b conj(Z_kb[f1][f2]) Gh_b[f1][f2]
// with Z_kb = F^*(w_k . u_b), Gh_b = F^*(dL/dy_b), N = N1 N2, and c_f2 = 1 at
// the DC and Nyquist columns (whose imaginary parts the inverse real
// transform discards after the column transform), 2 elsewhere.
// ===========================================================================

// Tiled transpose between natural [k][f1][f2] (f2 contiguous) and internal
// [k][f2][f1] (f1 contiguous), with a scale per f2 column.
template <bool TO_INTERNAL>
__global__ __launch_bounds__(256) void k_transpose_spec(const float2* __restrict__ src, float2* __restrict__ dst,
                                                        int N1, int H2, int scale_mode, float inv_n) {
  __shared__ float2 tile[32][33];
  const int k = blockIdx.z;
  const int64_t plane = (int64_t)N1 * H2;
  // tile origin: a = f1 block, b = f2 block
  const int a0 = blockIdx.y * 32, b0 = blockIdx.x * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 32 x 8
  for (int i = ty; i < 32; i += 8) {
    const int f1 = a0 + i, f2 = b0 + tx;       // natural: read/write along f2
    const int g1 = a0 + tx, g2 = b0 + i;       // internal: read/write along f1
    if (TO_INTERNAL) {
      if (f1 < N1 && f2 < H2) tile[i][tx] = src[k * plane + (int64_t)f1 * H2 + f2];
    } else {
      if (g1 < N1 && g2 < H2) tile[tx][i] = src[k * plane + (int64_t)g2 * N1 + g1];
    }
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int f1 = a0 + i, f2 = b0 + tx;
    const int g1 = a0 + tx, g2 = b0 + i;
    if (TO_INTERNAL) {
      if (g1 < N1 && g2 < H2) dst[k * plane + (int64_t)g2 * N1 + g1] = tile[tx][i];
    } else if (f1 < N1 && f2 < H2) {
      float2 v = tile[i][tx];
      if (scale_mode) {
        const float c = (f2 == 0 || f2 == H2 - 1) ? inv_n : 2.f * inv_n;  // DC and Nyquist columns
        v = cscale(v, c);
      }
      dst[k * plane + (int64_t)f1 * H2 + f2] = v;
    }
  }
}

// E_k[f2][:] = sum_b conj(colFFT(a_k1 . RA_k2[b][f2][:])) . Gh[b][f2][:], one
// (column, term) per FFT slot.
template <int L1>
__global__ __launch_bounds__(ffts_per_block(L1) * fft_threads(L1)) void k_grad2d_cols(
    const float2* __restrict__ RA, int64_t q_stride, const float2* __restrict__ Gh, int64_t batch, int H2, int m1,
    int m2, int dense, const float* __restrict__ wrows, float2* __restrict__ E, const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(L1), T = L1 / P, NF = ffts_per_block(L1);
  __shared__ float2 lds[NF * lds_len<L1>()];
  __shared__ float2 twl[L1];
  stage_twiddles<L1>(twl, tw);
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int nblk = (H2 + NF - 1) / NF;
  const int f2raw = blockIdx.x * NF + c;
  const bool valid = f2raw < H2;
  const int f2 = valid ? f2raw : H2 - 1;
  const int k = blockIdx.y;
  (void)nblk;
  const int k1 = dense ? 0 : k / m2, q = dense ? k : k % m2;
  (void)m1;
  const int64_t plane = (int64_t)L1 * H2;
  float2* my = lds + c * lds_len<L1>();
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  for (int64_t b = 0; b < batch; ++b) {
    const float2* col = RA + q * q_stride + b * plane + (int64_t)f2 * L1;
    const float2* gcol = Gh + b * plane + (int64_t)f2 * L1;
    float2 v[P], gv[P];
#pragma unroll
    for (int e = 0; e < P; ++e) {
      v[e] = col[t + T * e];
      gv[e] = gcol[t + T * e];
      if (!dense) v[e] = cscale(v[e], wrows[(int64_t)k1 * L1 + t + T * e]);
    }
    fft_wg<L1, P, false>(v, my, twl, t);
#pragma unroll
    for (int e = 0; e < P; ++e) acc[e] = cfma_conj(acc[e], v[e], gv[e]);
  }
  if (valid) {
    float2* dst = E + (int64_t)k * plane + (int64_t)f2 * L1;
#pragma unroll
    for (int e = 0; e < P; ++e) dst[t + T * e] = acc[e];
  }
}

template <int L1>
static LaunchStatus grad2d_cols_t(const Plan2D& p, int64_t batch, int64_t q_stride, float2* E, hipStream_t s) {
  constexpr int NF = ffts_per_block(L1), T = fft_threads(L1);
  const int nblk = (p.H2 + NF - 1) / NF;
  hipLaunchKernelGGL(k_grad2d_cols<L1>, dim3((unsigned)nblk, (unsigned)p.m), dim3(NF * T), 0, s, p.RA, q_stride,
                     p.Tws, batch, p.H2, p.m1, p.m2, p.dense ? 1 : 0, p.wrows, E, p.tw1);
  return hipGetLastError();
}

LaunchStatus launch_spectra2d(const Plan2D& p, const float2* in, float2* out, bool import, hipStream_t s) {
  const dim3 grid((unsigned)((p.H2 + 31) / 32), (unsigned)((p.N1 + 31) / 32), (unsigned)p.m);
  if (import)
    hipLaunchKernelGGL(k_transpose_spec<true>, grid, dim3(256), 0, s, in, const_cast<float2*>(p.Hs), p.N1, p.H2, 0,
                       1.f);
  else
    hipLaunchKernelGGL(k_transpose_spec<false>, grid, dim3(256), 0, s, p.Hs, out, p.N1, p.H2, 0, 1.f);
  return hipGetLastError();
}

LaunchStatus launch_grad2d(const Plan2D& p, const float* u, const float* gy, float2* gspec, int64_t batch,
                           float2* E, hipStream_t s, Tracer* tr) {
  const int64_t plane = (int64_t)p.N1 * p.H2;
  const int64_t q_stride = plane * batch;
  const int nq = p.dense ? p.m : p.m2;
  LaunchStatus e = rows_fwd(p.N2, u, p.N1, batch, p.wcols, p.dense ? RW_DENSE : RW_FACTOR, nq, p.RA, q_stride,
                            p.tw2, s, tr);
  if (e != hipSuccess) return e;
  e = rows_fwd(p.N2, gy, p.N1, batch, nullptr, RW_NONE, 1, p.Tws, q_stride, p.tw2, s, tr);
  if (e != hipSuccess) return e;
  e = cols_fft(p.N1, p.Tws, p.H2, batch, p.tw1, s, tr);
  if (e != hipSuccess) return e;
  {
    TraceScope ts(tr, "grad2d_cols", s);
    switch (p.N1) {
#define PC_CASE(LL)                                      \
  case LL:                                               \
    e = grad2d_cols_t<LL>(p, batch, q_stride, E, s);     \
    break;
      PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
      default:
        return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  const dim3 grid((unsigned)((p.H2 + 31) / 32), (unsigned)((p.N1 + 31) / 32), (unsigned)p.m);
  hipLaunchKernelGGL(k_transpose_spec<false>, grid, dim3(256), 0, s, E, gspec, p.N1, p.H2, 1,
                     1.0f / ((float)p.N1 * (float)p.N2));
  return hipGetLastError();
}

}  // namespace pc
