// 2D kernels of the convolution-product expansion on an N1 x N2 periodic
// image (row-major, N2 contiguous); the higher-dimensional extension of
// section 6.2 with index pairs taken modulo (N1, N2).
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
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

#include "fft_engine.hpp"
#include "pc_internal.hpp"

namespace pc {

#define PC_FOR_EACH_L2(X) \
  X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192) \
  X(96) X(192) X(384) X(768) X(1536) X(3072) X(6144)

// Window applied by the row kernels.  RW_BOX: one term whose window is the
// product of a row factor and a column factor, wsrc = [a[N1] | b[L2]]; the
// row kernels run it as RW_FACTOR on b, times a[r] per row.
enum RowWin { RW_NONE = 0, RW_FACTOR = 1, RW_DENSE = 2, RW_BOX = 3 };

// Device-memory access through the job tables' pointers.  The compiler
// cannot tell that a pointer read from a table addresses global memory and
// emits flat instructions for it, whose completion the hardware tracks on
// the same counter as LDS reads: every LDS wait of a transform then also
// waits for them.  These helpers read and write through global-address-space
// views (every table pointer addresses device memory).
typedef float pc_f2 __attribute__((ext_vector_type(2)));
#define PC_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ float2 gld(const float2* p, int64_t i) {
  const pc_f2 v = ((const PC_GLOBAL pc_f2*)p)[i];
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gst(float2* p, int64_t i, float2 v) { ((PC_GLOBAL pc_f2*)p)[i] = pc_f2{v.x, v.y}; }
__device__ __forceinline__ float gldf(const float* p, int64_t i) { return ((const PC_GLOBAL float*)p)[i]; }
typedef float pc_f4 __attribute__((ext_vector_type(4)));
// two consecutive complex entries (16 bytes, 16-byte aligned)
__device__ __forceinline__ float4 gld2(const float2* p, int64_t i) {
  const pc_f4 v = *(const PC_GLOBAL pc_f4*)(p + i);
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gst2(float2* p, int64_t i, float4 v) {
  *(PC_GLOBAL pc_f4*)(p + i) = pc_f4{v.x, v.y, v.z, v.w};
}

// Row tiles in LDS: column f of a tile holds the tile's 2G rows as G row
// pairs of 16 bytes; row pair rc sits at position rc ^ tile_swz(f), so that
// the lanes reading one row pair of 8 consecutive columns (one pass of a
// 16-byte access over the 32 banks) hit 8 different 16-byte slots
// (unswizzled, every column starts on the same bank).  G is a power of two;
// for G < 8 the swizzle takes column bits above the ones the row pairs
// already spread.
template <int G>
__device__ __forceinline__ int tile_swz(int f) {
  constexpr int SH = G >= 8 ? 0 : G == 4 ? 1 : G == 2 ? 2 : 3;
  return (f >> SH) & (G - 1);
}
template <int G>
__device__ __forceinline__ int tile_pos(int f, int rc) {
  return f * G + (rc ^ tile_swz<G>(f));
}
__device__ __forceinline__ void gstf(float* p, int64_t i, float v) { ((PC_GLOBAL float*)p)[i] = v; }

// The thread index, opaque to the compiler (an empty asm statement that
// claims to modify it).  Passed to a transform inside a runtime loop, it keeps
// the transform's per-element LDS addresses from being hoisted out of the
// loop, where they held up to 64 extra VGPRs for the whole loop and halved
// the waves per SIMD of these memory-bound passes; recomputing them costs a
// few integer instructions per iteration.
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// ---------------------------------------------------------------------------
// Launches are table-driven: every block reads a BlockRef (job, image,
// block, factor) and its job's descriptor, so one launch serves every
// instance whose transforms have the kernel's length, whatever their other
// dimension, term count or window format.  A single plan is the one-job case.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// row kernels: G row pairs (2G rows) per workgroup
// ---------------------------------------------------------------------------

// Row pairs per workgroup: as many as LDS allows (transform buffers plus the
// twiddle table within 156 KiB), at most 8 (tiles of 16 rows).
constexpr int row_pairs_per_block(int L2) {
  int g = 8;
  while (g > 1 && (g * (L2 + L2 / PAD) + L2) * 8 > 156 * 1024) g /= 2;
  return g;
}

// Per-row-pair LDS region of the row-forward pass: the transform's buffer,
// padded so that consecutive regions start 32 / G four-byte banks apart (of
// 32): the 8-byte reads of one column's G row pairs, 16 lanes per pass,
// then hit distinct banks.
template <int L2, int G>
constexpr int row_slot_len() {
  constexpr int len = lds_len<L2>(), want = (16 / G) % 16;
  return len + (want - len % 16 + 16) % 16;
}

// Orders the accesses of one transform slot to its own LDS region: a
// wavefront barrier when the slot's T threads lie in one wavefront (whose
// LDS operations complete in program order), else a workgroup barrier.
template <int T>
__device__ __forceinline__ void slot_sync() {
  if constexpr (T <= 64 && 64 % T == 0)
    wave_sync();
  else
    __syncthreads();
}

// Row pairs per workgroup of the small-tile variant.
constexpr int row_pairs_small(int L2) { return row_pairs_per_block(L2) < 2 ? row_pairs_per_block(L2) : 2; }

// Half-spectra of windowed rows, transposed: sout[q][img][f2][n1], f2 < H2.
// The body of a row-forward block bm (G row pairs, G * T threads), with the
// workgroup's LDS (G * row_slot_len<L2, G>() entries) and the staged
// twiddles; the per-length kernel and the persistent batch kernel both run
// it.
template <int L2, int G>
__device__ __forceinline__ void rows_fwd_body(const RowJob* __restrict__ jobs, const BlockRef bm,
                                              const float* __restrict__ x_arg, float2* __restrict__ lds,
                                              float2* __restrict__ twl, const float2* __restrict__ tw,
                                              const int tid) {
  constexpr int P = points_per_thread(L2), T = L2 / P, H2 = L2 / 2 + 1;
  constexpr int NT = G * T;
  TwStage<L2, NT> ts;
  ts.load(tw, tid);
  const RowJob& jb = jobs[bm.job];
  const int N1 = jb.N1;
  const float* x = jb.xp ? *jb.xp : (jb.x ? jb.x : x_arg);
  const int c = tid / T, t = tid % T;
  const int64_t img = bm.img;
  const int r0 = bm.blk * 2 * G;
  const int r = r0 + 2 * c;
  const int q = bm.q;
  // rows r and r + 1 of the job's image; columns n2 >= wrap read at n2 - gN2
  const float *ra, *rb;
  int wrap = L2;
  if (jb.gN2 > 0) {
    int ia = jb.g1 + r;  // g1 < gN1 and r + 1 < N1 <= gN1: one wrap at most
    if (ia >= jb.gN1) ia -= jb.gN1;
    const int ib = ia + 1 == jb.gN1 ? 0 : ia + 1;
    ra = x + (img * jb.gN1 + ia) * jb.gN2 + jb.g2;
    rb = x + (img * jb.gN1 + ib) * jb.gN2 + jb.g2;
    wrap = jb.gN2 - jb.g2;
  } else {
    ra = x + (img * N1 + r) * L2;
    rb = ra + L2;
  }
  float2 v[P];
  // masked rows and columns count as zero and are not read (the window box
  // of a section, the gradient's box of the output gradient)
  const bool la = jb.mrows <= 0 || r < jb.mrows, lb = jb.mrows <= 0 || r + 1 < jb.mrows;
  const int mc = jb.mcols > 0 ? jb.mcols : L2;
  int mode = jb.mode;
  const float* ws = jb.wsrc;
  float sa = 1.f, sb = 1.f;
  if (mode == RW_BOX) {
    sa = gldf(ws, r);
    sb = gldf(ws, r + 1);
    ws += N1;
    mode = RW_FACTOR;
  }
  // every load is issued unconditionally, masked samples at the row's first
  // address (lane 0's line: no extra traffic), then zeroed by a select; one
  // branch per window mode around straight-line code (a branch per element
  // made the compiler wait for each element's loads in turn)
  float xa[P], xb[P];
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int n2 = t + T * e;
    const int o = n2 < mc ? (n2 < wrap ? n2 : n2 - jb.gN2) : 0;
    xa[e] = gldf(ra, o);
    xb[e] = gldf(rb, o);
  }
  if (mode == RW_DENSE) {
    const float* wp = ws + ((int64_t)q * N1 + r) * L2;
    float wa[P], wb[P];
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int n2 = t + T * e < mc ? t + T * e : 0;
      wa[e] = gldf(wp, n2);
      wb[e] = gldf(wp, L2 + n2);
    }
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const bool in = t + T * e < mc;
      v[e] = make_float2(in && la ? wa[e] * xa[e] : 0.f, in && lb ? wb[e] * xb[e] : 0.f);
    }
  } else if (mode == RW_FACTOR) {
    const float* wp = ws + (int64_t)q * L2;
    float w[P];
#pragma unroll
    for (int e = 0; e < P; ++e) w[e] = gldf(wp, t + T * e < mc ? t + T * e : 0);
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const bool in = t + T * e < mc;
      v[e] = make_float2(in && la ? sa * w[e] * xa[e] : 0.f, in && lb ? sb * w[e] * xb[e] : 0.f);
    }
  } else {
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const bool in = t + T * e < mc;
      v[e] = make_float2(in && la ? xa[e] : 0.f, in && lb ? xb[e] : 0.f);
    }
  }
  constexpr int SL = row_slot_len<L2, G>();
  float2* my = lds + c * SL;
  ts.commit(twl, tid);
  fft_wv<L2, P, false, SYNC_WAVE>(v, my, twl, t);
  // the packed spectrum C of the slot's two rows into its own region (the
  // transform's last reads of it were this slot's own)
  slot_sync<T>();
#pragma unroll
  for (int e = 0; e < P; ++e) my[lpad(t + T * e)] = v[e];
  __syncthreads();
  // transposed output in 16-byte chunks: chunk ch is column f = ch / G of
  // row pair rc = ch mod G, separated from that pair's C as
  // U_a = (C[f] + conj C[-f]) / 2, U_b = (C[f] - conj C[-f]) / (2 i);
  // every LDS read first, then the stores (a read-store loop waited for each
  // read in turn)
  constexpr int CH = H2 * G, PT = (CH + NT - 1) / NT;
  float4 sv[PT];
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int ch = tid + i * NT;
    if (ch < CH) {
      const int f = ch / G;
      const float2* m = lds + (ch % G) * SL;
      const float2 cf = m[lpad(f)];
      const float2 cm = m[lpad(f == 0 ? 0 : L2 - f)];
      sv[i] = make_float4(0.5f * (cf.x + cm.x), 0.5f * (cf.y - cm.y), 0.5f * (cf.y + cm.y), -0.5f * (cf.x - cm.x));
    }
  }
  float2* o = jb.sout + (int64_t)q * jb.q_stride + img * ((int64_t)H2 * N1) + r0;
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int ch = tid + i * NT;
    if (ch < CH) gst2(o, (int64_t)(ch / G) * N1 + 2 * (ch % G), sv[i]);
  }
}

template <int L2, int G = row_pairs_per_block(L2)>
__global__ __launch_bounds__(G * fft_threads(L2)) void k_rows_fwd(
    const RowJob* __restrict__ jobs, const BlockRef* __restrict__ bmap, const float* __restrict__ x_arg,
    const float2* __restrict__ tw, int64_t img_limit) {
  static_assert((G * row_slot_len<L2, G>() + L2) * sizeof(float2) <= 160 * 1024, "row-forward LDS");
  __shared__ __attribute__((aligned(16))) float2 lds[G * row_slot_len<L2, G>()];
  __shared__ float2 twl[L2];
  const BlockRef bm = bmap[blockIdx.x];
  if (bm.img >= img_limit) return;  // uniform over the workgroup
  rows_fwd_body<L2, G>(jobs, bm, x_arg, lds, twl, tw, threadIdx.x);
}

// The transposed tile (f < L2/2 + 1, tile_pos layout) of a plane whose
// rows r0 .. r0 + 2G start at src (row stride N1 entries), copied straight
// from global memory into LDS (global_load_lds_dwordx4: no registers, no
// wait per load): each lane moves one row pair of one column, 16 bytes
// whose global address is 16-byte aligned (N1, r0 and the plane offsets
// even), the lanes of a wave to consecutive LDS positions.
template <int L2, int G>
__device__ __forceinline__ void tile_to_lds(const float2* __restrict__ src, int N1, float2* lds, int tid) {
  constexpr int T = fft_threads(L2), NT = G * T, CH = (L2 / 2 + 1) * G;
  // WL lanes per wave (a workgroup of fewer than 64 threads is one partial
  // wave; otherwise NT is a multiple of 64), NW waves
  constexpr int WL = NT < 64 ? NT : 64, NW = NT / WL, IT = (CH + NT - 1) / NT;
  static_assert(NW * WL == NT, "row workgroups are whole waves or one partial wave");
  const int w = tid / WL, lane = tid % WL;
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const int c0 = (j * NW + w) * WL;  // the wave's first chunk: its LDS destination
    const int ch = c0 + lane;
    if (ch < CH) {
      // LDS position ch holds column f's row pair (ch mod G) ^ tile_swz(f)
      // (ch >= 0 and the offset within the plane below 2^32: unsigned
      // 32-bit arithmetic)
      const unsigned f = (unsigned)ch / G, r = 2 * (((unsigned)ch % G) ^ tile_swz<G>((int)f));
      __builtin_amdgcn_global_load_lds((const PC_GLOBAL void*)(src + (f * (unsigned)N1 + r)),
                                       (__attribute__((address_space(3))) void*)(lds + 2 * c0), 16, 0, 0);
    }
  }
}

// One plane's tile (in LDS, tile_pos layout) of a row-inverse block:
// inverse row transforms of the G row pairs, the window of plane q applied
// and added to acc (thread t of slot c: row pair r, columns t + T e).
template <int L2, int G>
__device__ __forceinline__ void rows_inv_plane(const RowJob& jb, const int q, const int mode, const float* ws,
                                               const int r, const float4* tl, float2* my, const float2* twl,
                                               const int c, const int t, float2 (&acc)[points_per_thread(L2)]) {
  constexpr int P = points_per_thread(L2), T = L2 / P, H2 = L2 / 2 + 1;
  const int N1 = jb.N1;
  float2 v[P];
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int f = t + T * e;
    float2 a, b;
    if (f < H2) {
      const float4 ab = tl[tile_pos<G>(f, c)];
      a = make_float2(ab.x, ab.y);
      b = make_float2(ab.z, ab.w);
      if (f == 0 || f == L2 / 2) {  // the inverse real transform ignores these imaginary parts
        a.y = 0.f;
        b.y = 0.f;
      }
    } else {
      const float4 ab = tl[tile_pos<G>(L2 - f, c)];
      a = make_float2(ab.x, -ab.y);
      b = make_float2(ab.z, -ab.w);
    }
    v[e] = make_float2(a.x - b.y, a.y + b.x);  // a + i b
  }
  fft_wv<L2, P, true, SYNC_WAVE_ENTRY>(v, my, twl, opaque(t));
  // one branch per window mode around straight-line loads
  if (mode == RW_DENSE) {
    const float* wp = ws + ((int64_t)q * N1 + r) * L2 + t;
    float wa[P], wb[P];
#pragma unroll
    for (int e = 0; e < P; ++e) {
      wa[e] = gldf(wp, T * e);
      wb[e] = gldf(wp, L2 + T * e);
    }
#pragma unroll
    for (int e = 0; e < P; ++e) {
      acc[e].x = fmaf(wa[e], v[e].x, acc[e].x);
      acc[e].y = fmaf(wb[e], v[e].y, acc[e].y);
    }
  } else if (mode == RW_FACTOR) {
    const float* wp = ws + (int64_t)q * L2 + t;
    float w[P];
#pragma unroll
    for (int e = 0; e < P; ++e) w[e] = gldf(wp, T * e);
#pragma unroll
    for (int e = 0; e < P; ++e) {
      acc[e].x = fmaf(w[e], v[e].x, acc[e].x);
      acc[e].y = fmaf(w[e], v[e].y, acc[e].y);
    }
  } else {
#pragma unroll
    for (int e = 0; e < P; ++e) {
      acc[e].x += v[e].x;
      acc[e].y += v[e].y;
    }
  }
}

// The block's rows r, r + 1 (sums acc of thread t), scaled, to the output.
template <int L2>
__device__ __forceinline__ void rows_inv_store(const RowJob& jb, float* __restrict__ yout, const int64_t img,
                                               const int r, const int t, const float sa, const float sb,
                                               const float2 (&acc)[points_per_thread(L2)]) {
  constexpr int P = points_per_thread(L2), T = L2 / P;
  if (jb.oN2 > 0) {
    // section evaluation: the leading orows x ocols block goes straight to
    // its place in the output image (both axes wrapped)
    int ia = jb.o1 + r;
    if (ia >= jb.oN1) ia -= jb.oN1;
    const int ib = ia + 1 == jb.oN1 ? 0 : ia + 1;
    float* oa = yout + (img * jb.oN1 + ia) * jb.oN2;
    float* ob = yout + (img * jb.oN1 + ib) * jb.oN2;
    const bool wa = r < jb.orows, wb = r + 1 < jb.orows;
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int n2 = t + T * e;
      int o = jb.o2 + n2;
      if (o >= jb.oN2) o -= jb.oN2;
      if (n2 < jb.ocols) {
        if (wa) gstf(oa, o, acc[e].x * sa);
        if (wb) gstf(ob, o, acc[e].y * sb);
      }
    }
    return;
  }
  // columns n2 < ocols only (0: all)
  const int sc = jb.ocols > 0 ? jb.ocols : L2;
  float* oa = yout + (img * jb.N1 + r) * L2;
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int n2 = t + T * e;
    if (n2 < sc) {
      gstf(oa, n2, acc[e].x * sa);
      gstf(oa, n2 + L2, acc[e].y * sb);
    }
  }
}

// Real rows from transposed half-spectra:
// y[img][n1][n2] = scale * sum_{q < nq} w_q . rowIFFT(sin[q][img][:, n1]).
// PIPE: plane q + 1's tile is loaded into registers while plane q is
// transformed (latency hidden inside the workgroup, for a tile's share of
// registers per thread; see rows_inv_pipe for when that pays).  ONE: every
// job of the launch has one plane (nq = 1), so no sum is carried across a
// transform (fewer registers, one more wave per SIMD at 384 points).
template <int L2, int G, bool PIPE, bool ONE = false>
__device__ __forceinline__ void rows_inv_body(const RowJob* __restrict__ jobs, const BlockRef bm,
                                              float* __restrict__ y_arg, float2* __restrict__ lds,
                                              float2* __restrict__ twl, const float2* __restrict__ tw,
                                              float* __restrict__ rfac, const int tid) {
  constexpr int P = points_per_thread(L2), T = L2 / P, H2 = L2 / 2 + 1;
  constexpr int NT = G * T;
  TwStage<L2, NT> ts;
  ts.load(tw, tid);
  const RowJob& jb = jobs[bm.job];
  const int N1 = jb.N1;
  float* yout = jb.yp ? *jb.yp : (jb.y ? jb.y : y_arg);
  const int c = tid / T, t = tid % T;
  const int64_t img = bm.img;
  const int r0 = bm.blk * 2 * G;
  const int r = r0 + 2 * c;
  float2* my = lds + c * lds_len<L2>();
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  // the tile: H2 columns of G row pairs (tile_pos layout)
  constexpr int CH = H2 * G, PER = PIPE ? (CH + NT - 1) / NT : 1;
  const float2* src0 = jb.sin + img * ((int64_t)H2 * N1) + r0;
  float4* tl = reinterpret_cast<float4*>(lds);
  float4 nxt[PER];
  // LDS position ch of the tile holds column ch / G's row pair
  // (ch mod G) ^ tile_swz(column)
  auto tile_src = [&](int ch) { return (int64_t)(ch / G) * N1 + 2 * ((ch % G) ^ tile_swz<G>(ch / G)); };
  const int mode = jb.mode == RW_BOX ? RW_FACTOR : jb.mode;
  const float* ws = jb.mode == RW_BOX ? jb.wsrc + N1 : jb.wsrc;
  if constexpr (PIPE) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int ch = tid + i * NT;
      if (ch < CH) nxt[i] = gld2(src0, tile_src(ch));
    }
  }
  // a factored window's row factors, staged in LDS (visible after the
  // loop's first barrier) so that no register holds them across the transforms
  const bool box = jb.mode == RW_BOX;
  if (box && tid < 2 * G) rfac[tid] = gldf(jb.wsrc, r0 + tid);
  ts.commit(twl, tid);
  const int nq = ONE ? 1 : jb.nq;
  for (int q = 0; q < nq; ++q) {
    __syncthreads();  // the previous transform is done with LDS
    if constexpr (PIPE) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int ch = tid + i * NT;
        if (ch < CH) tl[ch] = nxt[i];
      }
      __syncthreads();
      if (q + 1 < nq) {
        const float2* src = src0 + (int64_t)(q + 1) * jb.q_stride;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
          const int ch = tid + i * NT;
          if (ch < CH) nxt[i] = gld2(src, tile_src(ch));
        }
      }
    } else {
      tile_to_lds<L2, G>(src0 + (int64_t)q * jb.q_stride, N1, lds, opaque(tid));
      __syncthreads();
    }
    rows_inv_plane<L2, G>(jb, q, mode, ws, r, tl, my, twl, c, t, acc);
  }
  const float sa = box ? rfac[2 * c] * jb.scale : jb.scale, sb = box ? rfac[2 * c + 1] * jb.scale : jb.scale;
  rows_inv_store<L2>(jb, yout, img, r, t, sa, sb, acc);
}

template <int L2, int G, bool PIPE, bool ONE = false>
__global__ __launch_bounds__(G * fft_threads(L2)) void k_rows_inv(
    const RowJob* __restrict__ jobs, const BlockRef* __restrict__ bmap, float* __restrict__ y_arg,
    const float2* __restrict__ tw, int64_t img_limit) {
  __shared__ __attribute__((aligned(16))) float2 lds[G * lds_len<L2>()];
  __shared__ float2 twl[L2];
  __shared__ float rfac[2 * G];
  const BlockRef bm = bmap[blockIdx.x];
  if (bm.img >= img_limit) return;  // uniform over the workgroup
  rows_inv_body<L2, G, PIPE, ONE>(jobs, bm, y_arg, lds, twl, tw, rfac, threadIdx.x);
}

// ---------------------------------------------------------------------------
// column kernels: NF columns per workgroup, each column contiguous
// ---------------------------------------------------------------------------

// Forward column pass for the term group bm.q: the group takes the column
// factors q in [q0, q1) and, for each, every row factor k1 (the column of
// src_q is loaded once and reused for all of them).  ngroups == 1: the
// inverse column transform of the sum is written to dst; otherwise the
// partial spectrum goes to part[group] for k_cols_sum_inv.
template <int L1, bool LATE, bool KEEP>
__device__ __forceinline__ void cols_fwd_body(const ColJob* __restrict__ jobs, const BlockRef bm,
                                              float2* __restrict__ lds, float2* __restrict__ twl,
                                              const float2* __restrict__ tw, const int tid) {
  constexpr int P = points_per_thread(L1), T = L1 / P, NF = ffts_per_block(L1);
  TwStage<L1, NF * T> ts;
  ts.load(tw, tid);
  const ColJob& jb = jobs[bm.job];
  const int H2 = jb.H2, m1 = jb.m1, m2 = jb.m2, dense = jb.dense, ngroups = jb.ngroups;
  const int c = tid / T, t = tid % T;
  const int64_t img = bm.img;
  const int f2raw = bm.blk * NF + c;
  const bool valid = f2raw < H2;
  const int f2 = valid ? f2raw : H2 - 1;  // idle slots recompute a valid column and store nothing
  const int64_t plane = (int64_t)L1 * H2;
  const int nq = dense ? m1 * m2 : m2;  // dense windows: q runs over all terms
  const int g = bm.q;
  const int q0 = (int)((int64_t)nq * g / ngroups), q1 = (int)((int64_t)nq * (g + 1) / ngroups);
  const int nk1 = dense ? 1 : m1;
  float2* my = lds + c * lds_len<L1>();
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  // elements e < ne of this thread are loaded (t + T e < nvalid_in), the
  // rest are zero
  const int nv = jb.nvalid_in == 0 ? L1 : jb.nvalid_in;
  const int ne = nv > t ? (nv - t + T - 1) / T : 0;
  float2 cv[P];
  auto load_col = [&](int q) {
    const float2* col = jb.src + q * jb.q_stride + img * plane + (int64_t)f2 * L1;
#pragma unroll
    for (int e = 0; e < P; ++e) cv[e] = e < ne ? gld(col, t + T * e) : make_float2(0.f, 0.f);
  };
  // the first column's loads go out before the twiddles are committed
  if (q0 < q1) load_col(q0);
  ts.commit(twl, tid);
  for (int q = q0; q < q1; ++q) {
    if (q > q0) load_col(q);
    for (int k1 = 0; k1 < nk1; ++k1) {
      const int k = dense ? q : k1 * m2 + q;
      const float2* Hk = jb.Hs + (int64_t)k * plane + (int64_t)f2 * L1;
      // the spectrum is loaded before the transform (its latency hides
      // behind it) or, LATE, after it (P fewer complex registers live across
      // the transform, which can buy another wave per SIMD)
      float2 hv[P], v[P];
      if constexpr (!LATE) {
#pragma unroll
        for (int e = 0; e < P; ++e) hv[e] = gld(Hk, t + T * e);
      }
      // row factor: loads issued together (a select per element would make
      // the compiler wait for each in turn)
      if (dense) {
#pragma unroll
        for (int e = 0; e < P; ++e) v[e] = cv[e];
      } else {
        float w[P];
#pragma unroll
        for (int e = 0; e < P; ++e) w[e] = gldf(jb.wrows, (int64_t)k1 * L1 + t + T * e);
#pragma unroll
        for (int e = 0; e < P; ++e) v[e] = cscale(cv[e], w[e]);
      }
      fft_wv<L1, P, false, SYNC_WAVE>(v, my, twl, opaque(t));
      if (KEEP && valid) {
        float2* kp = jb.keep + (int64_t)k * jb.keep_stride + img * plane + (int64_t)f2 * L1;
#pragma unroll
        for (int e = 0; e < P; ++e) gst(kp, t + T * e, v[e]);
      }
#pragma unroll
      for (int e = 0; e < P; ++e) acc[e] = cfma(acc[e], LATE ? gld(Hk, t + T * e) : hv[e], v[e]);
    }
  }
  if (ngroups == 1) {
    fft_wv<L1, P, true, SYNC_WAVE>(acc, my, twl, t);
    if (valid) {
      // rows t + T e < nvalid_out are stored (the rows the row-inverse pass reads)
      const int nvo = jb.nvalid_out == 0 ? L1 : jb.nvalid_out;
      const int no = nvo > t ? (nvo - t + T - 1) / T : 0;
      float2* dst = jb.dst + img * plane + (int64_t)f2 * L1;
#pragma unroll
      for (int e = 0; e < P; ++e)
        if (e < no) gst(dst, t + T * e, acc[e]);
    }
  } else if (valid) {
    float2* dst = jb.part + g * jb.part_stride + img * plane + (int64_t)f2 * L1;
#pragma unroll
    for (int e = 0; e < P; ++e) gst(dst, t + T * e, acc[e]);
  }
}

template <int L1, bool LATE, bool KEEP>
__global__ __launch_bounds__(ffts_per_block(L1) * fft_threads(L1)) void k_cols_fwd(
    const ColJob* __restrict__ jobs, const BlockRef* __restrict__ bmap, const float2* __restrict__ tw, int64_t img_limit) {
  constexpr int NF = ffts_per_block(L1);
  __shared__ float2 lds[NF * lds_len<L1>()];
  __shared__ float2 twl[L1];
  const BlockRef bm = bmap[blockIdx.x];
  if (bm.img >= img_limit) return;  // uniform over the workgroup
  cols_fwd_body<L1, LATE, KEEP>(jobs, bm, lds, twl, tw, threadIdx.x);
}

// dst[img][f2][:] = colIFFT(sum_g part[g][img][f2][:]).
template <int L1>
__global__ __launch_bounds__(ffts_per_block(L1) * fft_threads(L1)) void k_cols_sum_inv(
    const ColJob* __restrict__ jobs, const BlockRef* __restrict__ bmap, const float2* __restrict__ tw, int64_t img_limit) {
  constexpr int P = points_per_thread(L1), T = L1 / P, NF = ffts_per_block(L1);
  __shared__ float2 lds[NF * lds_len<L1>()];
  __shared__ float2 twl[L1];
  const BlockRef bm = bmap[blockIdx.x];
  if (bm.img >= img_limit) return;  // uniform over the workgroup
  stage_twiddles<L1>(twl, tw);
  const ColJob& jb = jobs[bm.job];
  const int H2 = jb.H2;
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int64_t img = bm.img;
  const int f2raw = bm.blk * NF + c;
  const bool valid = f2raw < H2;
  const int f2 = valid ? f2raw : H2 - 1;
  const int64_t off = img * ((int64_t)L1 * H2) + (int64_t)f2 * L1;
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = gld(jb.part, off + t + T * e);
  for (int g = 1; g < jb.ngroups; ++g) {
#pragma unroll
    for (int e = 0; e < P; ++e) acc[e] = cadd(acc[e], gld(jb.part, g * jb.part_stride + off + t + T * e));
  }
  fft_wv<L1, P, true, SYNC_WAVE>(acc, lds + c * lds_len<L1>(), twl, t);
  if (valid) {
#pragma unroll
    for (int e = 0; e < P; ++e) gst(jb.dst, off + t + T * e, acc[e]);
  }
}

// Adjoint column pass, one (column, q = bm.q) per FFT slot:
// dst_q[img][f2][:] = sum_k1 a_k1 . colIFFT(conj(H_k) . src[img][f2][:]),
// src column-transformed beforehand by k_cols_fft, or here when fft_src.
// PF: the next term's spectrum column is loaded before the current transform
// (its latency hides behind it, for P more complex registers).
template <int L1, bool PF>
__device__ __forceinline__ void cols_adj_body(const ColJob* __restrict__ jobs, const BlockRef bm,
                                              float2* __restrict__ lds, float2* __restrict__ twl,
                                              const float2* __restrict__ tw, const int tid) {
  constexpr int P = points_per_thread(L1), T = L1 / P, NF = ffts_per_block(L1);
  TwStage<L1, NF * T> ts;
  ts.load(tw, tid);
  const ColJob& jb = jobs[bm.job];
  const int H2 = jb.H2, m1 = jb.m1, m2 = jb.m2, dense = jb.dense;
  const int c = tid / T, t = tid % T;
  const int64_t img = bm.img;
  const int f2raw = bm.blk * NF + c;
  const bool valid = f2raw < H2;
  const int f2 = valid ? f2raw : H2 - 1;
  const int q = bm.q;
  const int64_t plane = (int64_t)L1 * H2;
  const int64_t coff = img * plane + (int64_t)f2 * L1;
  // elements e < ne of this thread are loaded (t + T e < nvalid_in), the
  // rest are zero
  const int nvi = jb.nvalid_in == 0 ? L1 : jb.nvalid_in;
  const int nei = nvi > t ? (nvi - t + T - 1) / T : 0;
  float2 vh[P];
#pragma unroll
  for (int e = 0; e < P; ++e) vh[e] = e < nei ? gld(jb.src, coff + t + T * e) : make_float2(0.f, 0.f);
  const int nk1 = dense ? 1 : m1;
  float2* my = lds + c * lds_len<L1>();
  ts.commit(twl, tid);
  if (jb.fft_src) fft_wv<L1, P, false, SYNC_WAVE>(vh, my, twl, t);  // uniform over the workgroup
  float2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
  // term k = k1 m2 + q (dense windows: k = q, one pass)
  const float2* Hq = jb.Hs + (int64_t)q * plane + (int64_t)f2 * L1;
  const int64_t k1_stride = (int64_t)m2 * plane;
  float2 hn[PF ? P : 1];
  if constexpr (PF) {
#pragma unroll
    for (int e = 0; e < P; ++e) hn[e] = gld(Hq, t + T * e);
  }
  for (int k1 = 0; k1 < nk1; ++k1) {
    float2 g[P];
    if constexpr (PF) {
#pragma unroll
      for (int e = 0; e < P; ++e) g[e] = cmulc(vh[e], hn[e]);
      if (k1 + 1 < nk1) {
        const float2* Hn = Hq + (int64_t)(k1 + 1) * k1_stride;
#pragma unroll
        for (int e = 0; e < P; ++e) hn[e] = gld(Hn, t + T * e);
      }
    } else {
      const float2* Hk = Hq + (int64_t)k1 * k1_stride;
#pragma unroll
      for (int e = 0; e < P; ++e) g[e] = cmulc(vh[e], gld(Hk, t + T * e));
    }
    fft_wv<L1, P, true, SYNC_WAVE>(g, my, twl, opaque(t));
    if (dense) {
#pragma unroll
      for (int e = 0; e < P; ++e) {
        acc[e].x += g[e].x;
        acc[e].y += g[e].y;
      }
    } else {
      float w[P];
#pragma unroll
      for (int e = 0; e < P; ++e) w[e] = gldf(jb.wrows, (int64_t)k1 * L1 + t + T * e);
#pragma unroll
      for (int e = 0; e < P; ++e) {
        acc[e].x = fmaf(w[e], g[e].x, acc[e].x);
        acc[e].y = fmaf(w[e], g[e].y, acc[e].y);
      }
    }
  }
  if (valid) {
    float2* dst = jb.dst + q * jb.q_stride + coff;
    // elements e < ne of this thread are stored (t + T e < nvalid_out)
    const int nv = jb.nvalid_out == 0 ? L1 : jb.nvalid_out;
    const int ne = nv > t ? (nv - t + T - 1) / T : 0;
#pragma unroll
    for (int e = 0; e < P; ++e)
      if (e < ne) gst(dst, t + T * e, acc[e]);
  }
}

template <int L1, bool PF>
__global__ __launch_bounds__(ffts_per_block(L1) * fft_threads(L1)) void k_cols_adj(
    const ColJob* __restrict__ jobs, const BlockRef* __restrict__ bmap, const float2* __restrict__ tw, int64_t img_limit) {
  constexpr int NF = ffts_per_block(L1);
  __shared__ float2 lds[NF * lds_len<L1>()];
  __shared__ float2 twl[L1];
  const BlockRef bm = bmap[blockIdx.x];
  if (bm.img >= img_limit) return;  // uniform over the workgroup
  cols_adj_body<L1, PF>(jobs, bm, lds, twl, tw, threadIdx.x);
}

// Column passes of single-term jobs (one term, one group: the sections of a
// sectioned plan, one-term plans), one column per FFT slot, with nothing
// carried across terms: forward dst = colIFFT(H . colFFT(a . src)), adjoint
// dst = a . colIFFT(conj(H) . colFFT(src)), a the row factor of a separable
// window (none for dense windows), rows n1 < nvalid_in read and
// n1 < nvalid_out written.  The spectrum column is loaded after the first
// transform.  KEEP (forward): the transformed windowed column U is also
// stored at keep[img][f2][:] for the backward pass.
template <int L1, bool ADJ, bool KEEP = false>
__global__ __launch_bounds__(ffts_per_block(L1) * fft_threads(L1)) void k_cols_1term(
    const ColJob* __restrict__ jobs, const BlockRef* __restrict__ bmap, const float2* __restrict__ tw,
    int64_t img_limit) {
  constexpr int P = points_per_thread(L1), T = L1 / P, NF = ffts_per_block(L1);
  __shared__ float2 lds[NF * lds_len<L1>()];
  __shared__ float2 twl[L1];
  const BlockRef bm = bmap[blockIdx.x];
  if (bm.img >= img_limit) return;  // uniform over the workgroup
  const int tid = threadIdx.x;
  TwStage<L1, NF * T> ts;
  ts.load(tw, tid);
  const ColJob& jb = jobs[bm.job];
  const int H2 = jb.H2;
  const int c = tid / T, t = tid % T;
  const int f2raw = bm.blk * NF + c;
  const bool valid = f2raw < H2;
  const int f2 = valid ? f2raw : H2 - 1;  // idle slots recompute a valid column and store nothing
  const int64_t coff = bm.img * ((int64_t)L1 * H2) + (int64_t)f2 * L1;
  const int nvi = jb.nvalid_in == 0 ? L1 : jb.nvalid_in;
  const int nvo = jb.nvalid_out == 0 ? L1 : jb.nvalid_out;
  const int nei = nvi > t ? (nvi - t + T - 1) / T : 0, neo = nvo > t ? (nvo - t + T - 1) / T : 0;
  float2 v[P];
#pragma unroll
  for (int e = 0; e < P; ++e) v[e] = e < nei ? gld(jb.src, coff + t + T * e) : make_float2(0.f, 0.f);
  if (!ADJ && !jb.dense) {  // the row factor of the windowed input
    float w[P];
#pragma unroll
    for (int e = 0; e < P; ++e) w[e] = gldf(jb.wrows, t + T * e);
#pragma unroll
    for (int e = 0; e < P; ++e) v[e] = cscale(v[e], w[e]);
  }
  float2* my = lds + c * lds_len<L1>();
  ts.commit(twl, tid);
  fft_wv<L1, P, false, SYNC_WAVE>(v, my, twl, opaque(t));
  if (KEEP && valid) {
    float2* kp = jb.keep + coff;
#pragma unroll
    for (int e = 0; e < P; ++e) gst(kp, t + T * e, v[e]);
  }
  const float2* Hk = jb.Hs + (int64_t)f2 * L1;
#pragma unroll
  for (int e = 0; e < P; ++e) v[e] = ADJ ? cmulc(v[e], gld(Hk, t + T * e)) : cmul(gld(Hk, t + T * e), v[e]);
  fft_wv<L1, P, true, SYNC_WAVE>(v, my, twl, opaque(t));
  if (ADJ && !jb.dense) {
    float w[P];
#pragma unroll
    for (int e = 0; e < P; ++e) w[e] = gldf(jb.wrows, t + T * e);
#pragma unroll
    for (int e = 0; e < P; ++e) v[e] = cscale(v[e], w[e]);
  }
  if (valid) {
    float2* dst = jb.dst + coff;
#pragma unroll
    for (int e = 0; e < P; ++e)
      if (e < neo) gst(dst, t + T * e, v[e]);
  }
}

// In-place column FFTs of dst: dst[img][f2][:] = colFFT(dst[img][f2][:]).
template <int L1>
__device__ __forceinline__ void cols_fft_body(const ColJob* __restrict__ jobs, const BlockRef bm,
                                              float2* __restrict__ lds, float2* __restrict__ twl,
                                              const float2* __restrict__ tw, const int tid) {
  constexpr int P = points_per_thread(L1), T = L1 / P, NF = ffts_per_block(L1);
  TwStage<L1, NF * T> ts;
  ts.load(tw, tid);
  const ColJob& jb = jobs[bm.job];
  const int H2 = jb.H2;
  const int c = tid / T, t = tid % T;
  const int64_t img = bm.img;
  const int f2raw = bm.blk * NF + c;
  const bool valid = f2raw < H2;
  const int f2 = valid ? f2raw : H2 - 1;
  const int64_t off = img * ((int64_t)L1 * H2) + (int64_t)f2 * L1;
  float2 v[P];
#pragma unroll
  for (int e = 0; e < P; ++e) v[e] = gld(jb.dst, off + t + T * e);
  ts.commit(twl, tid);
  fft_wv<L1, P, false, SYNC_WAVE>(v, lds + c * lds_len<L1>(), twl, t);
  if (valid) {
#pragma unroll
    for (int e = 0; e < P; ++e) gst(jb.dst, off + t + T * e, v[e]);
  }
}

template <int L1>
__global__ __launch_bounds__(ffts_per_block(L1) * fft_threads(L1)) void k_cols_fft(
    const ColJob* __restrict__ jobs, const BlockRef* __restrict__ bmap, const float2* __restrict__ tw, int64_t img_limit) {
  constexpr int NF = ffts_per_block(L1);
  __shared__ float2 lds[NF * lds_len<L1>()];
  __shared__ float2 twl[L1];
  const BlockRef bm = bmap[blockIdx.x];
  if (bm.img >= img_limit) return;  // uniform over the workgroup
  cols_fft_body<L1>(jobs, bm, lds, twl, tw, threadIdx.x);
}

// Backward column pass of a single-term job (the sections of Lemma 3.2):
// one column per FFT slot, all images in turn.  From one transform of the
// output gradient's column, V = colFFT(src), it forms the adjoint's plane
// colIFFT(conj(H) . V) (into dst, when want_gu) and the spectra gradient's
// column sum_b conj(U) . V, with U = colFFT(dst) (the row transforms of the
// windowed input left by the forward pass) or U read from keep.  dst is read
// before it is overwritten, column by column, by the same threads.
template <int L1>
__global__ __launch_bounds__(ffts_per_block(L1) * fft_threads(L1)) void k_cols_bwd1(
    const ColJob* __restrict__ jobs, const BlockRef* __restrict__ bmap, const float2* __restrict__ tw,
    float2* __restrict__ gext, int64_t img_limit) {
  constexpr int P = points_per_thread(L1), T = L1 / P, NF = ffts_per_block(L1);
  __shared__ float2 lds[NF * lds_len<L1>()];
  __shared__ float2 twl[L1];
  const BlockRef bm = bmap[blockIdx.x];
  stage_twiddles<L1>(twl, tw);
  const ColJob& jb = jobs[bm.job];
  const int H2 = jb.H2;
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int f2raw = bm.blk * NF + c;
  const bool valid = f2raw < H2;
  const int f2 = valid ? f2raw : H2 - 1;
  const int64_t plane = (int64_t)L1 * H2;
  float2* my = lds + c * lds_len<L1>();
  const float2* Hc = jb.Hs + (int64_t)f2 * L1;
  // per-thread element counts of the row ranges that matter
  auto count = [&](int nv) { return nv == 0 ? P : (nv > t ? (nv - t + T - 1) / T : 0); };
  const int ne_src = count(jb.nv_src), ne_in = count(jb.nvalid_in), ne_out = count(jb.nvalid_out);
  const int64_t nimg = jb.nimg < img_limit ? jb.nimg : img_limit;
  float2 ga[P];
#pragma unroll
  for (int e = 0; e < P; ++e) ga[e] = make_float2(0.f, 0.f);
  for (int64_t b = 0; b < nimg; ++b) {
    const int64_t coff = b * plane + (int64_t)f2 * L1;
    float2 v[P];
#pragma unroll
    for (int e = 0; e < P; ++e) v[e] = e < ne_src ? gld(jb.src, coff + t + T * e) : make_float2(0.f, 0.f);
    fft_wv<L1, P, false, SYNC_WAVE>(v, my, twl, opaque(t));
    if (jb.grad) {
      float2 z[P];
      if (jb.keep) {
#pragma unroll
        for (int e = 0; e < P; ++e) z[e] = gld(jb.keep, coff + t + T * e);
      } else {
#pragma unroll
        for (int e = 0; e < P; ++e) z[e] = e < ne_in ? gld(jb.dst, coff + t + T * e) : make_float2(0.f, 0.f);
        fft_wv<L1, P, false, SYNC_WAVE>(z, my, twl, opaque(t));
      }
#pragma unroll
      for (int e = 0; e < P; ++e) ga[e] = cfma_conj(ga[e], z[e], v[e]);
    }
    if (jb.want_gu) {
#pragma unroll
      for (int e = 0; e < P; ++e) v[e] = cmulc(v[e], gld(Hc, t + T * e));
      fft_wv<L1, P, true, SYNC_WAVE>(v, my, twl, opaque(t));
      if (valid) {
#pragma unroll
        for (int e = 0; e < P; ++e)
          if (e < ne_out) gst(jb.dst, coff + t + T * e, v[e]);
      }
    }
  }
  if (jb.grad && jb.gext_off >= 0) {  // uniform over the workgroup
    // the NF columns through LDS (stride L1 + 1: the lanes reading one row
    // of NF columns hit distinct banks), then rows of NF entries to the
    // natural layout, scaled
    static_assert(NF * (L1 + 1) <= NF * lds_len<L1>(), "LDS room for the gradient columns");
    if (!gext) return;  // uniform: no gradient wanted
    __syncthreads();  // every slot is done with its transform buffer
#pragma unroll
    for (int e = 0; e < P; ++e) lds[c * (L1 + 1) + t + T * e] = ga[e];
    __syncthreads();
    const int f20 = bm.blk * NF;
    float2* gn = gext + jb.gext_off;
    for (int idx = threadIdx.x; idx < NF * L1; idx += NF * T) {
      const int f1 = idx / NF, cc = idx % NF, g2 = f20 + cc;
      if (g2 < H2) {
        const float s = (g2 == 0 || g2 == H2 - 1) ? jb.ginv_n : 2.f * jb.ginv_n;
        gst(gn, (int64_t)f1 * H2 + g2, cscale(lds[cc * (L1 + 1) + f1], s));
      }
    }
  } else if (jb.grad && valid) {
    float2* gp = jb.grad + (int64_t)f2 * L1;
#pragma unroll
    for (int e = 0; e < P; ++e) gst(gp, t + T * e, ga[e]);
  }
}

// ---------------------------------------------------------------------------
// Persistent batch passes.  One launch per pass and length group runs the
// blocks of every transform length of the group; its workgroups
// (PERSIST_THREADS threads, row passes with G = PERSIST_THREADS / T row
// pairs) walk the item list with a grid stride, stage the item's twiddles and
// run the pass body.  The
// variants are fixed to the ones with the fewest registers (spectrum loaded
// after the transform, no prefetch, no pipelined row-inverse tiles): a
// launch holds the code of every length of its group, so its register count
// is the largest of them.
// ---------------------------------------------------------------------------
#define PC_FOR_EACH_PL(X) X(64) X(96) X(128) X(192) X(256) X(384) X(512)
// lengths by points per thread (8, 12, 16): one persistent launch per group,
// so each holds the code of lengths with similar register needs
#define PC_FOR_EACH_PG0(X) X(64) X(128)
#define PC_FOR_EACH_PG1(X) X(96) X(192) X(384)
#define PC_FOR_EACH_PG2(X) X(256) X(512)

template <int L>
constexpr int prow_pairs() { return PERSIST_THREADS / fft_threads(L); }

template <int KIND, int L>
constexpr int plds_entries() {
  // transform buffers, twiddles and (row-inverse) the 2G row factors
  return (KIND == PK_ROWS_FWD   ? prow_pairs<L>() * row_slot_len<L, prow_pairs<L>()>()
          : KIND == PK_ROWS_INV ? prow_pairs<L>() * lds_len<L>()
                                : ffts_per_block(L) * lds_len<L>()) +
         L + (KIND == PK_ROWS_INV ? prow_pairs<L>() : 0);
}

template <int KIND, int L>
__device__ __forceinline__ void persist_item(const PItem& w, float2* smem, const float* x_arg, float* y_arg) {
  float2* twl = smem;
  float2* lds = smem + L;
  // (each body stages the item's twiddles itself)
  // an opaque copy of the thread index: the body's per-element addresses are
  // recomputed per item instead of living across the item loop
  const int tid = opaque((int)threadIdx.x);
  if constexpr (KIND == PK_ROWS_FWD) {
    rows_fwd_body<L, prow_pairs<L>()>(static_cast<const RowJob*>(w.jobs), w.bm, x_arg, lds, twl, w.tw, tid);
  } else if constexpr (KIND == PK_ROWS_INV) {
    rows_inv_body<L, prow_pairs<L>(), false>(static_cast<const RowJob*>(w.jobs), w.bm, y_arg, lds, twl, w.tw,
                                             reinterpret_cast<float*>(lds + prow_pairs<L>() * lds_len<L>()), tid);
  } else if constexpr (KIND == PK_COLS_A) {
    if (w.sub == 0)
      cols_fwd_body<L, true, false>(static_cast<const ColJob*>(w.jobs), w.bm, lds, twl, w.tw, tid);
    else
      cols_fft_body<L>(static_cast<const ColJob*>(w.jobs), w.bm, lds, twl, w.tw, tid);
  } else {
    cols_adj_body<L, false>(static_cast<const ColJob*>(w.jobs), w.bm, lds, twl, w.tw, tid);
  }
}

template <int KIND, int PG>
__global__ __launch_bounds__(PERSIST_THREADS) void k_persist(const PItem* __restrict__ items, int n_items,
                                                            const float* __restrict__ x_arg, float* __restrict__ y_arg) {
  extern __shared__ __attribute__((aligned(16))) float2 smem[];
  // workgroup b takes items b, b + grid, b + 2 grid, ... of the list (longest
  // first): no shared counter, whose same-address atomics would serialise
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    __syncthreads();  // the previous item is done with LDS
    const PItem w = items[it];
#define PC_CASE(LL)                                  \
  case LL:                                           \
    persist_item<KIND, LL>(w, smem, x_arg, y_arg);   \
    break;
    if constexpr (PG == 0) {
      switch (w.L) { PC_FOR_EACH_PG0(PC_CASE) }
    } else if constexpr (PG == 1) {
      switch (w.L) { PC_FOR_EACH_PG1(PC_CASE) }
    } else {
      switch (w.L) { PC_FOR_EACH_PG2(PC_CASE) }
    }
#undef PC_CASE
  }
}

bool persist_length(int L) {
  switch (L) {
#define PC_CASE(LL) case LL:
    PC_FOR_EACH_PL(PC_CASE)
#undef PC_CASE
    return true;
  }
  return false;
}

int persist_group(int L) { return points_per_thread(L) == 8 ? 0 : points_per_thread(L) == 12 ? 1 : 2; }

int persist_block_rows(int L2) {
  switch (L2) {
#define PC_CASE(LL) \
  case LL:          \
    return 2 * prow_pairs<LL>();
    PC_FOR_EACH_PL(PC_CASE)
#undef PC_CASE
  }
  return 0;
}

template <int KIND>
static int plds_bytes_of(int L) {
  switch (L) {
#define PC_CASE(LL) \
  case LL:          \
    return plds_entries<KIND, LL>() * (int)sizeof(float2);
    PC_FOR_EACH_PL(PC_CASE)
#undef PC_CASE
  }
  return 0;
}

int persist_lds_bytes(int kind, const std::vector<int>& lengths) {
  int b = 0;
  for (int L : lengths) {
    const int x = kind == PK_ROWS_FWD   ? plds_bytes_of<PK_ROWS_FWD>(L)
                  : kind == PK_ROWS_INV ? plds_bytes_of<PK_ROWS_INV>(L)
                  : kind == PK_COLS_A   ? plds_bytes_of<PK_COLS_A>(L)
                                        : plds_bytes_of<PK_COLS_ADJ>(L);
    b = std::max(b, x);
  }
  return b;
}

template <int KIND>
static const void* persist_fn_k(int pg) {
  if (pg == 0) return reinterpret_cast<const void*>(k_persist<KIND, 0>);
  if (pg == 1) return reinterpret_cast<const void*>(k_persist<KIND, 1>);
  return reinterpret_cast<const void*>(k_persist<KIND, 2>);
}

static const void* persist_fn(int kind, int pg) {
  switch (kind) {
    case PK_ROWS_FWD: return persist_fn_k<PK_ROWS_FWD>(pg);
    case PK_COLS_A: return persist_fn_k<PK_COLS_A>(pg);
    case PK_COLS_ADJ: return persist_fn_k<PK_COLS_ADJ>(pg);
  }
  return persist_fn_k<PK_ROWS_INV>(pg);
}

// workgroups of a persistent launch: as many as the device holds at once
// (never more than the items)
int persist_grid(int kind, int pg, int lds_bytes, int64_t n_items) {
  int dev = 0, cus = 256, per_cu = 1;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_fn(kind, pg), PERSIST_THREADS, lds_bytes) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return (int)std::min<int64_t>(n_items, (int64_t)cus * per_cu);
}

// ---------------------------------------------------------------------------
// host side: block maps and launches
// ---------------------------------------------------------------------------
int row_block_rows(int L2, bool small) { return 2 * (small ? row_pairs_small(L2) : row_pairs_per_block(L2)); }
int col_block_cols(int L1) { return ffts_per_block(L1); }
int row_threads(int L2, bool small) {
  return (small ? row_pairs_small(L2) : row_pairs_per_block(L2)) * fft_threads(L2);
}
int col_threads(int L1) { return ffts_per_block(L1) * fft_threads(L1); }

void append_row_blocks(std::vector<BlockRef>& out, int job, int64_t n_img, int N1, int L2, int nq, bool small,
                       int rows, int block_rows) {
  const int br = block_rows > 0 ? block_rows : row_block_rows(L2, small);
  const int nb = rows > 0 && rows < N1 ? (rows + br - 1) / br : N1 / br;
  for (int64_t img = 0; img < n_img; ++img)
    for (int b = 0; b < nb; ++b)
      for (int q = 0; q < nq; ++q) out.push_back(BlockRef{job, (int)img, b, q});
}

void append_col_blocks(std::vector<BlockRef>& out, int job, int64_t n_img, int H2, int L1, int nsub) {
  const int nb = (H2 + col_block_cols(L1) - 1) / col_block_cols(L1);
  for (int64_t img = 0; img < n_img; ++img)
    for (int b = 0; b < nb; ++b)
      for (int q = 0; q < nsub; ++q) out.push_back(BlockRef{job, (int)img, b, q});
}

// Late loads pay where the early variant is down to two waves per SIMD and
// the late one has more (measured: the 1024 and 2048 column passes of single
// images, 1.6x faster).  With three or more waves, early loads are worth
// more when a launch's instances loop over several terms (each term's
// spectrum loads during the previous term's transform; measured on 256
// instances of 4 to 16 terms and 128 to 512 columns: late loads at 192, 256
// and 384 points cost 12%), and less when every instance has a single term,
// where there is no previous transform to hide behind (the 384-point
// single-term sections of C5: late loads 2% faster).
template <int L1>
static bool late_pays(bool multi_term) {
  const int threads = col_threads(L1);
  const int waves = (threads + 63) / 64;
  int early = 0, late = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&early, k_cols_fwd<L1, false, false>, threads, 0) != hipSuccess) return false;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&late, k_cols_fwd<L1, true, false>, threads, 0) != hipSuccess) return false;
  const int early_per_simd = early * waves / 4, late_per_simd = late * waves / 4;
  return late_per_simd > early_per_simd && (!multi_term || early_per_simd <= 2);
}

// The adjoint's prefetch pays wherever it costs no resident workgroup
// (measured: 2048^2, 64 terms, 2% faster; 128 to 512 columns, where it costs
// a wave per SIMD, 2% slower).
template <int L1>
static bool prefetch_pays() {
  const int threads = col_threads(L1);
  int plain = 0, pf = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&plain, k_cols_adj<L1, false>, threads, 0) != hipSuccess)
    return false;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pf, k_cols_adj<L1, true>, threads, 0) != hipSuccess) return false;
  return pf >= plain;
}

// One decision per length, cached.  (A tuning table entry, when the plan's
// workload has one, overrides these rules: see tune.cpp.)
template <class Decide>
static bool decide_once(std::map<int, bool>& known, std::mutex& mu, int L1, Decide decide) {
  std::lock_guard<std::mutex> g(mu);
  const auto it = known.find(L1);
  if (it != known.end()) return it->second;
  const bool r = decide(L1);
  known[L1] = r;
  return r;
}

bool cols_fwd_late(int L1, bool multi_term) {
  static std::mutex mu;
  static std::map<int, bool> known;
  return decide_once(known, mu, multi_term ? -L1 : L1, [](int key) {
    const bool b = key < 0;
    switch (b ? -key : key) {
#define PC_CASE(LL) \
  case LL:          \
    return late_pays<LL>(b);
      PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
    }
    return false;
  });
}

// The row-inverse pipeline pays where it keeps at least two waves per SIMD
// without spilling (measured: 256 instances of 128 to 512 points, 6% faster
// with it; the 2048-point rows of a single image, where it costs a wave per
// SIMD, 3% slower).
template <int L2, int G>
static bool pipe_pays() {
  const int threads = G * fft_threads(L2);
  const int waves = (threads + 63) / 64;
  int blocks = 0;
  hipFuncAttributes a{};
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_rows_inv<L2, G, true>, threads, 0) != hipSuccess)
    return false;
  if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_rows_inv<L2, G, true>)) != hipSuccess) return false;
  return blocks * waves / 4 >= 2 && a.localSizeBytes == 0;
}

bool rows_inv_pipe(int L2, bool small) {
  static std::mutex mu;
  static std::map<int, bool> known;
  return decide_once(known, mu, small ? -L2 : L2, [](int key) {
    const bool sm = key < 0;
    switch (sm ? -key : key) {
#define PC_CASE(LL) \
  case LL:          \
    return sm ? pipe_pays<LL, row_pairs_small(LL)>() : pipe_pays<LL, row_pairs_per_block(LL)>();
      PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
    }
    return false;
  });
}

bool cols_adj_prefetch(int L1) {
  static std::mutex mu;
  static std::map<int, bool> known;
  return decide_once(known, mu, L1, [](int L) {
    switch (L) {
#define PC_CASE(LL) \
  case LL:          \
    return prefetch_pays<LL>();
      PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
    }
    return false;
  });
}

int col_groups_for(int H2, int64_t batch, int nq) {
  // split the forward column pass over groups of column factors until about
  // sixteen column transforms per compute unit are launched: with two or
  // three resident workgroups per CU, fewer leave the last round of
  // workgroups mostly empty (measured: 2048^2, 64 terms, 8 -> 16 per CU cut
  // the pass by ~15%; 32 per CU was slower again from the partial sums)
  const int64_t cols = (int64_t)H2 * batch;
  const int64_t target = 256 * 16;
  int g = 1;
  while (g < nq && cols * g < target) g *= 2;
  return g < nq ? g : nq;
}

LaunchStatus launch_set(const LaunchSet& ls, int64_t nblocks, const float* x_arg, float* y_arg, hipStream_t s,
                        Tracer* tr, int64_t img_limit) {
  if (nblocks <= 0) return hipSuccess;
  if (ls.persist >= 0) {
    static const char* const names[] = {"persist_rows_fwd", "persist_cols_a", "persist_cols_adj", "persist_rows_inv"};
    TraceScope ts(tr, names[ls.persist & 3], s);
    const dim3 pg((unsigned)nblocks), pb(PERSIST_THREADS);
    const void* fn = persist_fn(ls.persist, ls.pgroup);
    void* args[] = {(void*)&ls.items, (void*)&ls.n_items, (void*)&x_arg, (void*)&y_arg};
    const hipError_t e = hipLaunchKernel(fn, pg, pb, args, (size_t)ls.lds_bytes, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
  }
  if (ls.kind == KK_SEC_SCATTER)  // (traced as sec_scatter by the launcher)
    return launch_sec_scatter(*ls.sec, nullptr, ls.sec_adjoint, nblocks < ls.sec->cap ? nblocks : ls.sec->cap, s, tr,
                              ls.sec_out);
  TraceScope ts(tr, kernel_kind_name(ls.kind), s);
  const dim3 grid((unsigned)nblocks), block((unsigned)ls.threads);
  const RowJob* rj = static_cast<const RowJob*>(ls.jobs);
  const ColJob* cj = static_cast<const ColJob*>(ls.jobs);
  switch (ls.kind) {
    case KK_ROWS_FWD:
      switch (ls.L) {
#define PC_CASE(LL) \
  case LL:          \
    if (ls.small_rows)  \
      hipLaunchKernelGGL((k_rows_fwd<LL, row_pairs_small(LL)>), grid, block, 0, s, rj, ls.bmap, x_arg, ls.tw, img_limit); \
    else  \
      hipLaunchKernelGGL(k_rows_fwd<LL>, grid, block, 0, s, rj, ls.bmap, x_arg, ls.tw, img_limit); \
    return hipGetLastError();
        PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
      }
      break;
    case KK_ROWS_INV:
      switch (ls.L) {
#define PC_CASE(LL) \
  case LL:          \
    if (ls.small_rows && ls.pipe)  \
      hipLaunchKernelGGL((k_rows_inv<LL, row_pairs_small(LL), true>), grid, block, 0, s, rj, ls.bmap, y_arg, ls.tw, img_limit); \
    else if (ls.small_rows && ls.one_plane)  \
      hipLaunchKernelGGL((k_rows_inv<LL, row_pairs_small(LL), false, true>), grid, block, 0, s, rj, ls.bmap, y_arg, ls.tw, img_limit); \
    else if (ls.small_rows)  \
      hipLaunchKernelGGL((k_rows_inv<LL, row_pairs_small(LL), false>), grid, block, 0, s, rj, ls.bmap, y_arg, ls.tw, img_limit); \
    else if (ls.pipe)  \
      hipLaunchKernelGGL((k_rows_inv<LL, row_pairs_per_block(LL), true>), grid, block, 0, s, rj, ls.bmap, y_arg, ls.tw, img_limit); \
    else if (ls.one_plane)  \
      hipLaunchKernelGGL((k_rows_inv<LL, row_pairs_per_block(LL), false, true>), grid, block, 0, s, rj, ls.bmap, y_arg, ls.tw, img_limit); \
    else  \
      hipLaunchKernelGGL((k_rows_inv<LL, row_pairs_per_block(LL), false>), grid, block, 0, s, rj, ls.bmap, y_arg, ls.tw, img_limit); \
    return hipGetLastError();
        PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
      }
      break;
    case KK_COLS_FWD:
      switch (ls.L) {
#define PC_CASE(LL) \
  case LL:          \
    if (ls.one && ls.keep)     \
      hipLaunchKernelGGL((k_cols_1term<LL, false, true>), grid, block, 0, s, cj, ls.bmap, ls.tw, img_limit); \
    else if (ls.one)           \
      hipLaunchKernelGGL((k_cols_1term<LL, false>), grid, block, 0, s, cj, ls.bmap, ls.tw, img_limit); \
    else if (ls.keep && ls.late)    \
      hipLaunchKernelGGL((k_cols_fwd<LL, true, true>), grid, block, 0, s, cj, ls.bmap, ls.tw, img_limit); \
    else if (ls.keep)          \
      hipLaunchKernelGGL((k_cols_fwd<LL, false, true>), grid, block, 0, s, cj, ls.bmap, ls.tw, img_limit); \
    else if (ls.late)          \
      hipLaunchKernelGGL((k_cols_fwd<LL, true, false>), grid, block, 0, s, cj, ls.bmap, ls.tw, img_limit); \
    else                       \
      hipLaunchKernelGGL((k_cols_fwd<LL, false, false>), grid, block, 0, s, cj, ls.bmap, ls.tw, img_limit); \
    return hipGetLastError();
        PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
      }
      break;
    case KK_COLS_SUM:
      switch (ls.L) {
#define PC_CASE(LL) \
  case LL:          \
    hipLaunchKernelGGL(k_cols_sum_inv<LL>, grid, block, 0, s, cj, ls.bmap, ls.tw, img_limit); \
    return hipGetLastError();
        PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
      }
      break;
    case KK_COLS_ADJ:
      switch (ls.L) {
#define PC_CASE(LL) \
  case LL:          \
    if (ls.one) \
      hipLaunchKernelGGL((k_cols_1term<LL, true>), grid, block, 0, s, cj, ls.bmap, ls.tw, img_limit); \
    else if (ls.prefetch) \
      hipLaunchKernelGGL((k_cols_adj<LL, true>), grid, block, 0, s, cj, ls.bmap, ls.tw, img_limit); \
    else \
      hipLaunchKernelGGL((k_cols_adj<LL, false>), grid, block, 0, s, cj, ls.bmap, ls.tw, img_limit); \
    return hipGetLastError();
        PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
      }
      break;
    case KK_COLS_BWD1:
      switch (ls.L) {
#define PC_CASE(LL) \
  case LL:          \
    hipLaunchKernelGGL(k_cols_bwd1<LL>, grid, block, 0, s, cj, ls.bmap, ls.tw, reinterpret_cast<float2*>(y_arg), img_limit); \
    return hipGetLastError();
        PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
      }
      break;
    case KK_COLS_FFT:
      switch (ls.L) {
#define PC_CASE(LL) \
  case LL:          \
    hipLaunchKernelGGL(k_cols_fft<LL>, grid, block, 0, s, cj, ls.bmap, ls.tw, img_limit); \
    return hipGetLastError();
        PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
      }
      break;
  }
  return hipErrorInvalidValue;
}

const char* kernel_kind_name(int kind) {
  switch (kind) {
    case KK_ROWS_FWD: return "rows_fwd";
    case KK_ROWS_INV: return "rows_inv";
    case KK_COLS_FWD: return "cols_fwd";
    case KK_COLS_SUM: return "cols_sum";
    case KK_COLS_ADJ: return "cols_adj";
    case KK_COLS_FFT: return "cols_fft";
    case KK_COLS_BWD1: return "cols_bwd";
    case KK_SEC_SCATTER: return "sec_scatter";
  }
  return "unknown";
}

// A single plan's launch with batch images: the block maps are image-major,
// so a smaller batch launches a prefix of the map.
static LaunchStatus run(const LaunchSet& ls, int64_t batch, const float* x, float* y, hipStream_t s, Tracer* tr) {
  return launch_set(ls, ls.blocks_per_img * batch, x, y, s, tr);
}

LaunchStatus launch_spec2d(const Plan2D& p, const float* h, hipStream_t s) {
  LaunchStatus e = launch_set(p.spec_rows, p.spec_rows.blocks, h, nullptr, s, nullptr);
  if (e != hipSuccess) return e;
  return launch_set(p.spec_cols, p.spec_cols.blocks, nullptr, nullptr, s, nullptr);
}

LaunchStatus launch_fwd2d(const Plan2D& p, const float* u, float* y, int64_t batch, hipStream_t s, Tracer* tr,
                          bool keep) {
  LaunchStatus e = run(p.fwd_rows, batch, u, nullptr, s, tr);
  if (e == hipSuccess) e = run(keep && p.keep ? p.fwd_cols_keep : p.fwd_cols, batch, nullptr, nullptr, s, tr);
  if (e == hipSuccess && p.col_groups > 1) e = run(p.fwd_sum, batch, nullptr, nullptr, s, tr);
  if (e == hipSuccess) e = run(p.fwd_rows_out, batch, nullptr, y, s, tr);
  return e;
}

// The adjoint's tail after launch_grad2d left V = colFFT(rowFFT(v)) in Tws
// (plans with more than one term, whose adjoint column pass takes V).
LaunchStatus launch_adj2d_tail(const Plan2D& p, float* x, int64_t batch, hipStream_t s, Tracer* tr) {
  LaunchStatus e = run(p.adj_cols, batch, nullptr, nullptr, s, tr);
  if (e == hipSuccess) e = run(p.adj_rows_out, batch, nullptr, x, s, tr);
  return e;
}

LaunchStatus launch_adj2d(const Plan2D& p, const float* v, float* x, int64_t batch, hipStream_t s, Tracer* tr) {
  LaunchStatus e = run(p.adj_rows, batch, v, nullptr, s, tr);
  if (e == hipSuccess && !p.adj_fused) e = run(p.adj_fft, batch, nullptr, nullptr, s, tr);
  if (e == hipSuccess) e = run(p.adj_cols, batch, nullptr, nullptr, s, tr);
  if (e == hipSuccess) e = run(p.adj_rows_out, batch, nullptr, x, s, tr);
  return e;
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
// [k][f2][f1] (f1 contiguous), with a scale per f2 column.  A tile is TA
// frequencies f1 by TB frequencies f2; the natural rows (N2/2+1 entries) start
// at any 8-byte offset, so the cache lines at a tile's two f2 edges are shared
// with its neighbours.  The tiles of one f1 strip take consecutive indices and
// xcd_major keeps consecutive indices on one XCD, so those shared lines meet
// in one L2 instead of reaching HBM as partial writes from two.
constexpr int SPEC_TA = 32, SPEC_TB = 32, SPEC_THREADS = 256;
template <bool TO_INTERNAL>
__global__ __launch_bounds__(SPEC_THREADS) void k_transpose_spec(const float2* __restrict__ src,
                                                                float2* __restrict__ dst, int N1, int H2,
                                                                int scale_mode, float inv_n, int64_t nblocks) {
  constexpr int TA = SPEC_TA, TB = SPEC_TB;
  __shared__ float2 tile[TA][TB + 1];
  const int nbB = (H2 + TB - 1) / TB, nbA = (N1 + TA - 1) / TA;
  const int64_t b = xcd_major(blockIdx.x, nblocks);
  const int jb = (int)(b % nbB);
  const int64_t rest = b / nbB;
  const int ib = (int)(rest % nbA);
  const int64_t k = rest / nbA;
  const int64_t plane = (int64_t)N1 * H2;
  const int a0 = ib * TA, b0 = jb * TB;
  src += k * plane;
  dst += k * plane;
  // natural side: lanes run along f2; internal side: lanes run along f1;
  // every load of the thread issued before the tile is written
  constexpr int PER = TA * TB / SPEC_THREADS;
  static_assert(PER * SPEC_THREADS == TA * TB, "whole tiles per thread count");
  float2 tv[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int idx = (int)threadIdx.x + r * SPEC_THREADS;
    const int i = TO_INTERNAL ? idx / TB : idx % TA, j = TO_INTERNAL ? idx % TB : idx / TA;
    if (a0 + i < N1 && b0 + j < H2)
      tv[r] = TO_INTERNAL ? src[(int64_t)(a0 + i) * H2 + b0 + j] : src[(int64_t)(b0 + j) * N1 + a0 + i];
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int idx = (int)threadIdx.x + r * SPEC_THREADS;
    const int i = TO_INTERNAL ? idx / TB : idx % TA, j = TO_INTERNAL ? idx % TB : idx / TA;
    if (a0 + i < N1 && b0 + j < H2) tile[i][j] = tv[r];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < TA * TB; idx += SPEC_THREADS) {
    if (TO_INTERNAL) {
      const int i = idx % TA, j = idx / TA;
      if (a0 + i < N1 && b0 + j < H2) dst[(int64_t)(b0 + j) * N1 + a0 + i] = tile[i][j];
    } else {
      const int i = idx / TB, j = idx % TB;
      const int f2 = b0 + j;
      if (a0 + i < N1 && f2 < H2) {
        float2 v = tile[i][j];
        if (scale_mode) {
          const float c = (f2 == 0 || f2 == H2 - 1) ? inv_n : 2.f * inv_n;  // DC and Nyquist columns
          v = cscale(v, c);
        }
        dst[(int64_t)(a0 + i) * H2 + f2] = v;
      }
    }
  }
}

// Launches the transpose over all m terms, in groups of terms small enough
// for one grid (at most 2^22 workgroups per launch).
template <bool TO_INTERNAL>
static LaunchStatus transpose_spec(const Plan2D& p, const float2* src, float2* dst, int scale_mode, float inv_n,
                                   hipStream_t s) {
  const int64_t per_term = (int64_t)((p.N1 + SPEC_TA - 1) / SPEC_TA) * ((p.H2 + SPEC_TB - 1) / SPEC_TB);
  const int64_t group = std::max<int64_t>(1, ((int64_t)1 << 22) / per_term);
  const int64_t plane = (int64_t)p.N1 * p.H2;
  for (int64_t k0 = 0; k0 < p.m; k0 += group) {
    const int64_t nb = std::min<int64_t>(group, p.m - k0) * per_term;
    hipLaunchKernelGGL(k_transpose_spec<TO_INTERNAL>, dim3((unsigned)nb), dim3(SPEC_THREADS), 0, s,
                       src + k0 * plane, dst + k0 * plane, p.N1, p.H2, scale_mode, inv_n, nb);
  }
  return hipGetLastError();
}

// E_k[f2][:] = sum_b conj(colFFT(a_k1 . RA_k2[b][f2][:])) . Gh[b][f2][:].
// One (column, column factor k2) per FFT slot, looping over the row factors
// k1 (dense windows: one term per slot): the terms of one k2 share the
// columns of RA_k2 and Gh, which then come from the caches instead of being
// fetched by a separate workgroup per term.  Gh is read after the transform:
// nothing of it lives across the transform, which lowers the register count
// at every length (2048: 177 -> 155 VGPRs, a third wave per SIMD).
template <int L1>
__global__ __launch_bounds__(ffts_per_block(L1) * fft_threads(L1)) void k_grad2d_cols(
    const float2* __restrict__ RA, int64_t q_stride, const float2* __restrict__ Gh, int64_t batch, int H2, int m1,
    int m2, int dense, const float* __restrict__ wrows, float2* __restrict__ E, const float2* __restrict__ tw,
    const float2* __restrict__ keep, int64_t keep_stride) {
  constexpr int P = points_per_thread(L1), T = L1 / P, NF = ffts_per_block(L1);
  __shared__ float2 lds[NF * lds_len<L1>()];
  __shared__ float2 twl[L1];
  stage_twiddles<L1>(twl, tw);
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int nblk = (H2 + NF - 1) / NF;
  const int f2raw = blockIdx.x * NF + c;
  const bool valid = f2raw < H2;
  const int f2 = valid ? f2raw : H2 - 1;
  const int q = blockIdx.y;  // column factor (dense: the term)
  (void)nblk;
  const int nk1 = dense ? 1 : m1;
  const int64_t plane = (int64_t)L1 * H2;
  float2* my = lds + c * lds_len<L1>();
  for (int k1 = 0; k1 < nk1; ++k1) {
    const int k = dense ? q : k1 * m2 + q;
    float2 acc[P];
#pragma unroll
    for (int e = 0; e < P; ++e) acc[e] = make_float2(0.f, 0.f);
    for (int64_t b = 0; b < batch; ++b) {
      const float2* col = RA + q * q_stride + b * plane + (int64_t)f2 * L1;
      const float2* gcol = Gh + b * plane + (int64_t)f2 * L1;
      float2 v[P];
      if (keep) {  // U_k kept by the forward pass (uniform over the workgroup)
        const float2* kp = keep + (int64_t)k * keep_stride + b * plane + (int64_t)f2 * L1;
#pragma unroll
        for (int e = 0; e < P; ++e) v[e] = kp[t + T * e];
      } else {
#pragma unroll
        for (int e = 0; e < P; ++e) v[e] = col[t + T * e];
        if (!dense) {
          float w[P];
#pragma unroll
          for (int e = 0; e < P; ++e) w[e] = wrows[(int64_t)k1 * L1 + t + T * e];
#pragma unroll
          for (int e = 0; e < P; ++e) v[e] = cscale(v[e], w[e]);
        }
        fft_wv<L1, P, false, SYNC_WAVE>(v, my, twl, opaque(t));
      }
#pragma unroll
      for (int e = 0; e < P; ++e) acc[e] = cfma_conj(acc[e], v[e], gcol[t + T * e]);
    }
    if (valid) {
      float2* dst = E + (int64_t)k * plane + (int64_t)f2 * L1;
#pragma unroll
      for (int e = 0; e < P; ++e) dst[t + T * e] = acc[e];
    }
  }
}

template <int L1>
static LaunchStatus grad2d_cols_t(const Plan2D& p, int64_t batch, int64_t q_stride, float2* E, const float2* keep,
                                  hipStream_t s) {
  constexpr int NF = ffts_per_block(L1), T = fft_threads(L1);
  const int nblk = (p.H2 + NF - 1) / NF;
  hipLaunchKernelGGL(k_grad2d_cols<L1>, dim3((unsigned)nblk, (unsigned)(p.dense ? p.m : p.m2)), dim3(NF * T), 0, s,
                     p.RA, q_stride,
                     p.Tws, batch, p.H2, p.m1, p.m2, p.dense ? 1 : 0, p.wrows, E, p.tw1, keep,
                     q_stride);
  return hipGetLastError();
}

int64_t transpose_blocks(int N1, int H2) {
  return (int64_t)((N1 + SPEC_TA - 1) / SPEC_TA) * ((H2 + SPEC_TB - 1) / SPEC_TB);
}

// One workgroup per tile of one job's plane (the job found by a binary
// search over the jobs' first workgroups); tiles as in k_transpose_spec.
__global__ __launch_bounds__(SPEC_THREADS) void k_transpose_tab(const TransposeJob* __restrict__ jobs, int njobs,
                                                               float2* __restrict__ ext, int to_internal) {
  constexpr int TA = SPEC_TA, TB = SPEC_TB;
  __shared__ float2 tile[TA][TB + 1];
  const int64_t blk = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (jobs[mid].block0 <= blk) lo = mid; else hi = mid - 1;
  }
  const TransposeJob jb = jobs[lo];
  const int N1 = jb.N1, H2 = jb.H2;
  const int nbB = (H2 + TB - 1) / TB;
  const int64_t b = blk - jb.block0;
  const int a0 = (int)(b / nbB) * TA, b0 = (int)(b % nbB) * TB;
  float2* nat = ext + jb.ext_off;
  // every load of the thread issued before the tile is written
  constexpr int PER = TA * TB / SPEC_THREADS;
  static_assert(PER * SPEC_THREADS == TA * TB, "whole tiles per thread count");
  float2 tv[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int idx = (int)threadIdx.x + r * SPEC_THREADS;
    const int i = to_internal ? idx / TB : idx % TA, j = to_internal ? idx % TB : idx / TA;
    if (a0 + i < N1 && b0 + j < H2)
      tv[r] = to_internal ? gld(nat, (int64_t)(a0 + i) * H2 + b0 + j) : gld(jb.internal, (int64_t)(b0 + j) * N1 + a0 + i);
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int idx = (int)threadIdx.x + r * SPEC_THREADS;
    const int i = to_internal ? idx / TB : idx % TA, j = to_internal ? idx % TB : idx / TA;
    if (a0 + i < N1 && b0 + j < H2) tile[i][j] = tv[r];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < TA * TB; idx += SPEC_THREADS) {
    if (to_internal) {
      const int i = idx % TA, j = idx / TA;
      if (a0 + i < N1 && b0 + j < H2) gst(jb.internal, (int64_t)(b0 + j) * N1 + a0 + i, tile[i][j]);
    } else {
      const int i = idx / TB, j = idx % TB;
      const int f2 = b0 + j;
      if (a0 + i < N1 && f2 < H2) {
        float2 v = tile[i][j];
        if (jb.scale_mode) v = cscale(v, (f2 == 0 || f2 == H2 - 1) ? jb.inv_n : 2.f * jb.inv_n);
        gst(nat, (int64_t)(a0 + i) * H2 + f2, v);
      }
    }
  }
}

LaunchStatus launch_transpose_set(const TransposeSet& ts, float2* ext, bool to_internal, hipStream_t s) {
  if (ts.blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_tab, dim3((unsigned)ts.blocks), dim3(SPEC_THREADS), 0, s, ts.jobs, ts.njobs, ext,
                     to_internal ? 1 : 0);
  return hipGetLastError();
}

LaunchStatus launch_spectra2d(const Plan2D& p, const float2* in, float2* out, bool import, hipStream_t s) {
  if (import) return transpose_spec<true>(p, in, const_cast<float2*>(p.Hs), 0, 1.f, s);
  return transpose_spec<false>(p, p.Hs, out, 0, 1.f, s);
}

LaunchStatus launch_grad2d(const Plan2D& p, const float* u, const float* gy, float2* gspec, int64_t batch,
                           float2* E, hipStream_t s, Tracer* tr, bool rows_u, const float2* keep) {
  const int64_t plane = (int64_t)p.N1 * p.H2;
  const int64_t q_stride = plane * p.batch_cap;
  LaunchStatus e = hipSuccess;
  if (rows_u && !keep) e = run(p.fwd_rows, batch, u, nullptr, s, tr);  // RA_q = rowFFT(b_q . u)
  if (e != hipSuccess) return e;
  e = run(p.adj_rows, batch, gy, nullptr, s, tr);              // Tws = rowFFT(gy)
  if (e != hipSuccess) return e;
  e = run(p.adj_fft, batch, nullptr, nullptr, s, tr);          // Tws = colFFT(Tws)
  if (e != hipSuccess) return e;
  {
    TraceScope ts(tr, "grad2d_cols", s);
    switch (p.N1) {
#define PC_CASE(LL)                                      \
  case LL:                                               \
    e = grad2d_cols_t<LL>(p, batch, q_stride, E, keep, s); \
    break;
      PC_FOR_EACH_L2(PC_CASE)
#undef PC_CASE
      default:
        return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  return transpose_spec<false>(p, E, gspec, 1, 1.0f / ((float)p.N1 * (float)p.N2), s);
}

}  // namespace pc
