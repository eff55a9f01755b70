// Internal interfaces between the plan runtime (pc_api.cpp) and the kernel
// translation units.  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace pc {

// Launch status: hipSuccess, or hipErrorInvalidValue for a size with no
// instantiated kernel (the plan checks sizes first, so that is a bug).
using LaunchStatus = hipError_t;

// Points per thread used for an FFT of length L (3-smooth lengths need a
// multiple of 3).
constexpr int points_per_thread(int L) {
  return (L % 3 == 0) ? (L >= 1536 ? 24 : 12) : (L >= 256 ? 16 : 8);
}
constexpr int fft_threads(int L) { return L / points_per_thread(L); }
// FFTs per workgroup for the batched row / column kernels.
constexpr int ffts_per_block(int L) {
  int t = fft_threads(L);
  int nf = 256 / t;
  return nf < 1 ? 1 : nf;
}

bool fft_size_supported(int64_t L);  // 64..8192, 2^a or 3*2^a

// The chip deals workgroups to its 8 XCDs round-robin (workgroup b to XCD
// b % 8), each XCD with its own L2.  xcd_major renumbers a launch so that
// every XCD receives one contiguous range of the returned indices (identity
// when the launch is not a multiple of 8 workgroups): workgroups that read
// the same data, given neighbouring indices, then share one L2.
constexpr int XCDS = 8;
__device__ __forceinline__ int64_t xcd_major(int64_t b, int64_t nblocks) {
  if (nblocks % XCDS) return b;
  return (b % XCDS) * (nblocks / XCDS) + b / XCDS;
}

// Optional per-kernel timing: the launchers bracket every kernel with
// begin/end (HIP events recorded on the launch stream).
struct Tracer {
  virtual void begin(const char* kernel, hipStream_t s) = 0;
  virtual void end(hipStream_t s) = 0;
  virtual ~Tracer() = default;
};

struct TraceScope {
  Tracer* t;
  hipStream_t s;
  TraceScope(Tracer* tr, const char* name, hipStream_t st) : t(tr), s(st) {
    if (t) t->begin(name, s);
  }
  ~TraceScope() {
    if (t) t->end(s);
  }
};

// --------------------------------------------------------------------------
// 1D, N <= 8192: everything for one signal pair in one workgroup
// --------------------------------------------------------------------------
struct Small1D {
  int L;                     // N
  int m;
  const float* w;            // m x L windows
  const float2* H;           // m x L full complex spectra, natural order
  const float2* tw;          // engine twiddles for L
};
LaunchStatus launch_spec1d_full(int L, const float* h, float2* H, int m, const float2* tw, hipStream_t s);
LaunchStatus launch_fwd1d_small(const Small1D& p, const float* u, float* y, int64_t batch, hipStream_t s,
                                Tracer* tr = nullptr);
LaunchStatus launch_adj1d_small(const Small1D& p, const float* v, float* x, int64_t batch, hipStream_t s,
                                Tracer* tr = nullptr);

// --------------------------------------------------------------------------
// 1D, N = R * L (four-step): inner length L in a workgroup, R classes
// --------------------------------------------------------------------------
// Position of element f2 = t + T e inside an L-long block of the four-step
// path (T = L / P threads, e < P): elements e and e + 1 of thread t are
// adjacent, (e / 2) 2T + 2t + e % 2.
__host__ __device__ constexpr int block_pos(int f2, int T) {
  return ((f2 / T) >> 1) * (2 * T) + 2 * (f2 % T) + ((f2 / T) & 1);
}

struct Large1D {
  int L, R;                  // N = R * L
  int P;                     // points per thread of the inner transform (plan-time choice)
  int m;
  const float* wc;           // compacted window values, concatenated
  const int* w_off;          // m: support start (mod N)
  const int* w_len;          // m: support length (0 = empty window)
  const int64_t* w_base;     // m: start of window k inside wc
  const float2* Hd;          // m x R x L, Hd[k][f1][block_pos(f2)] = H_k[f] W_N^{f o_k}, f = f1 + R f2
  const float2* cw;          // short supports: m x R x chunks x L,
                             // cw[k][f1][c][block_pos(d)] = w_k[o_k + c L + d] W_N^{f1 (c L + d)}
  const float2* tw;          // engine twiddles for L
  const float2* twN;         // exp(-2 i pi j / N), j < N
  const float2* twC;         // class table: twC[f1 * L + n2] = exp(-2 i pi f1 n2 / N)
  const float* zeros;        // N zeros: the second signal of a pair when there is none
  int chunks;                // short supports: every window support is at most chunks x L long
                             // (1 or 2); 0: long-support path
  // adjoint work items: long path, (term, chunk of at most L samples of its
  // support); short supports, one per term (chunk 0, the whole support)
  int n_items;
  const int* item_k;
  const int* item_d0;        // chunk start inside the term's support
  const int* item_oc;        // chunk origin on the circle
  const int* item_len;       // item length (<= L, or <= chunks x L on the short-support path)
  const int64_t* item_out;   // offset of the item's samples in a pair's P block
  int64_t p_stride;          // float2 per pair in the P block
  // overlap-add: items that can cover each tile of 256 samples (CSR)
  const int* tile_off;       // N/256 + 1 entries
  const int* tile_items;
  // workspaces
  float2* Bws;               // pairs x R x L (block layout)
  float2* Vws;               // pairs x R x L (block layout)
  float2* Pws;               // pairs x p_stride
};
bool fourstep_variant_supported(int L, int R, int P);
LaunchStatus launch_fold_fft(const Large1D& p, const float* xa, int64_t n_sig, float2* out, bool pairs, hipStream_t s,
                             Tracer* tr = nullptr);
// out[i] = conj(in[i]), i < n (in may equal out)
LaunchStatus launch_conj(const float2* in, float2* out, int64_t n, hipStream_t s);
// Hd (natural frame, m x R x L) -> window-origin frame, in place
LaunchStatus launch_origin_phase1d(const Large1D& p, float2* Hd, hipStream_t s);
LaunchStatus launch_fwd1d_large(const Large1D& p, const float* u, float* y, int64_t batch, hipStream_t s,
                                Tracer* tr = nullptr);
LaunchStatus launch_adj1d_large(const Large1D& p, const float* v, float* x, int64_t batch, hipStream_t s,
                                Tracer* tr = nullptr);

// --------------------------------------------------------------------------
// 2D, N1 x N2 (row-major, N2 contiguous), half spectra N1 x (N2/2 + 1)
// --------------------------------------------------------------------------

// One instance of a row pass (row transforms of length N2).
struct RowJob {
  const float* x;      // input images (row-forward); null: the launch's pointer argument
  float* y;            // output images (row-inverse); null: the launch's pointer argument
  const float* wsrc;   // window source (see RowWin in the 2D kernels)
  int mode;            // 0 none, 1 column factors b_q[n2], 2 dense windows w_q[n1][n2],
                       // 3 one term's row and column factors [a[N1] | b[N2]]
  int N1;              // rows per image
  int nq;              // row-inverse: factor planes accumulated
  float scale;         // row-inverse: output scale
  const float2* sin;   // row-inverse: input planes [q][img][f2][n1]
  float2* sout;        // row-forward: output planes [q][img][f2][n1]
  int64_t q_stride;    // elements between factor planes
  // row-forward, section evaluation (gN2 > 0): the job's image img is the
  // box of image img of the launch's input (gN1 x gN2 samples) whose origin
  // is (g1, g2), both axes wrapped; needs N1 <= gN1, L2 <= gN2, g1 < gN1,
  // g2 < gN2
  int gN1 = 0, gN2 = 0, g1 = 0, g2 = 0;
  // batches: the input (row-forward) or output (row-inverse) pointer is read
  // from this device table entry at run time, so that each call can name
  // new buffers; null: x / y / the launch's pointer argument
  const float* const* xp = nullptr;
  float* const* yp = nullptr;
  // row-forward: samples of rows r >= mrows or columns n2 >= mcols read as
  // zero (0: no mask); the section gradient's box of the output gradient
  int mrows = 0, mcols = 0;
  // row-inverse, section evaluation (oN2 > 0): row r < orows of the job's
  // image img is written, columns n2 < ocols only, to image img of the output
  // (oN1 x oN2 samples) at ((o1 + r) mod oN1, (o2 + n2) mod oN2); with
  // oN2 == 0, ocols > 0 limits the stored columns of every row
  int oN1 = 0, oN2 = 0, o1 = 0, o2 = 0, orows = 0, ocols = 0;
};

// One instance of a column pass (column transforms of length N1).
struct ColJob {
  const float2* src;   // input planes
  float2* dst;         // output planes (in place for the transform-only pass)
  float2* part;        // partial sums of the forward pass (ngroups > 1)
  const float2* Hs;    // spectra, m planes [k][f2][f1]
  const float* wrows;  // row-axis window factors a_k1[n1] (separable)
  int64_t q_stride;    // between factor planes of src (forward) / dst (adjoint)
  int64_t part_stride;
  int H2, m1, m2, dense, ngroups;
  // adjoint pass of a single-term job: transform src's columns first, in
  // registers (no separate k_cols_fft pass and plane round trip)
  int fft_src = 0;
  // rows of the columns known to matter (0: all N1): both passes read src
  // entries n1 < nvalid_in only (the rest are zero: rows the row pass
  // skipped) and write dst entries n1 < nvalid_out only (the rest are never
  // read)
  int nvalid_in = 0, nvalid_out = 0;
  // forward pass: when keep is set, the transformed windowed column of term
  // k is also stored at keep[k * keep_stride + img * plane + f2 * N1] (the
  // windowed spectra U_k kept for the backward pass)
  float2* keep = nullptr;
  int64_t keep_stride = 0;
  // backward pass of a single-term job (k_cols_bwd1): src = row transforms
  // of the output gradient (rows < nv_src matter), dst = row transforms of
  // the windowed input (rows < nvalid_in; U_k read from keep instead when
  // set), overwritten with the adjoint's planes (rows < nvalid_out) when
  // want_gu; grad (optional) receives sum over the images of conj(U_k) V,
  // one plane [f2][f1]; nimg images.  With gext_off >= 0 that sum goes
  // instead, scaled by c(f2) ginv_n (c = 1 at f2 = 0 and f2 = H2 - 1, else
  // 2), to the launch's gradient buffer at gext_off + f1 H2 + f2 (the
  // section's spectrum in its natural layout); grad then only flags it.
  float2* grad = nullptr;
  int64_t gext_off = -1;
  float ginv_n = 0.f;
  int want_gu = 1;
  int nv_src = 0;
  int64_t nimg = 1;
};

// Block of a table-driven launch: job, image, block within the image,
// factor or term group.
struct BlockRef {
  int job, img, blk, q;
};

enum KernelKind { KK_ROWS_FWD = 0, KK_ROWS_INV, KK_COLS_FWD, KK_COLS_SUM, KK_COLS_ADJ, KK_COLS_FFT, KK_COLS_BWD1, KK_SEC_SCATTER };

// Persistent batch passes: every row or column block of a pass, whatever
// its transform length (within a length group), is one work item of one
// launch; the workgroups walk the list with a grid stride.
enum PersistKind { PK_ROWS_FWD = 0, PK_COLS_A = 1, PK_COLS_ADJ = 2, PK_ROWS_INV = 3 };
struct PItem {
  const void* jobs;  // device RowJob[] or ColJob[] of the item's length
  BlockRef bm;
  const float2* tw;  // engine twiddles for L
  int L;
  int sub;           // PK_COLS_A: 0 forward column pass, 1 column transform of V
};
constexpr int PERSIST_THREADS = 256;
// transform lengths the persistent kernels hold code for
bool persist_length(int L);
// rows per block of the persistent row passes (G = PERSIST_THREADS / T row pairs)
int persist_block_rows(int L2);
// dynamic LDS bytes of a persistent pass over the given lengths
int persist_lds_bytes(int kind, const std::vector<int>& lengths);
// length group of a persistent launch (points per thread 8, 12, 16)
int persist_group(int L);
int persist_grid(int kind, int pg, int lds_bytes, int64_t n_items);

// A prepared launch: kernel kind and length, device tables, block counts.
struct Sec2D;

struct LaunchSet {
  int kind = 0;
  int L = 0;
  int threads = 0;
  const void* jobs = nullptr;      // device RowJob[] or ColJob[]
  const BlockRef* bmap = nullptr;  // device
  int64_t blocks = 0;              // blocks of the whole table
  int64_t blocks_per_img = 0;      // single plans: blocks per image (prefix launches)
  const float2* tw = nullptr;      // engine twiddles for L
  bool small_rows = false;         // row kernels: the small-tile variant (row_block_rows(L, true) rows)
  bool late = false;               // forward column kernel: the late-spectrum variant (cols_fwd_late)
  bool prefetch = false;           // adjoint column kernel: the prefetching variant (cols_adj_prefetch)
  bool pipe = false;               // row-inverse kernel: the pipelined variant (rows_inv_pipe)
  bool one_plane = false;          // row-inverse kernel: every job sums one plane (its ONE variant)
  bool keep = false;               // forward column kernel: the variant storing U_k (jobs' keep pointers)
  bool one = false;                // column kernels: every job single-term (k_cols_1term)
  // persistent pass (persist >= 0: a PersistKind) of length group pgroup:
  // items (device PItem[]), their count and the dynamic LDS bytes
  int persist = -1;
  int pgroup = 0;
  const PItem* items = nullptr;
  int n_items = 0;
  int lds_bytes = 0;
  // overlap-add of a sectioned plan in a batch (KK_SEC_SCATTER): its section
  // geometry, the direction, and the batch table entry holding the output
  const Sec2D* sec = nullptr;
  bool sec_adjoint = false;
  float* const* sec_out = nullptr;
};

struct Plan2D {
  int N1, N2, H2;            // H2 = N2/2 + 1
  int m, m1, m2;             // separable: m = m1*m2, term k = k1*m2 + k2; dense: m1 = 1, m2 = m
  bool dense;                // dense windows m x N1 x N2 (or, wmode 3, one term's two factors)
  int wmode;                 // the row passes' window mode (1 separable, 2 dense, 3 factored single term)
  int64_t batch_cap;         // images the workspaces hold
  const float* wrows;        // separable: m1 x N1 (factor along rows, a_k1[n1])
  const float* wcols;        // separable: m2 x N2 (factor along columns, b_k2[n2]); dense: m x N1 x N2;
                             // wmode 3: a[N1] then b[N2]
  const float2* Hs;          // m planes, column-major: Hs[k][f2][f1]
  const float2* tw1;         // engine twiddles for N1
  const float2* tw2;         // engine twiddles for N2
  float2* RA;                // nq x batch_cap planes (nq = m2 or m), column-major [f2][n1]
  float2* Tws;               // batch_cap planes
  int col_groups;            // term groups of the forward column pass
  bool adj_fused;            // single term: adj_cols transforms its input itself (adj_fft unused by the adjoint)
  float2* Part;              // col_groups x batch_cap planes of partial spectra (col_groups > 1)
  LaunchSet fwd_rows, fwd_cols, fwd_sum, fwd_rows_out;
  LaunchSet fwd_cols_keep;   // fwd_cols storing U_k into keep (when the plan keeps them)
  float2* keep = nullptr;    // m x batch_cap planes of U_k, or null
  LaunchSet adj_rows, adj_fft, adj_cols, adj_rows_out;
  LaunchSet spec_rows, spec_cols;
};

int col_groups_for(int H2, int64_t batch, int nq);

// ---------------------------------------------------------------------------
// Tuning table (tune.cpp): measured choices of the per-length variants for
// given workloads, overriding the rules above.  A workload is named by a
// 64-bit key of its plan description (or, for a batch, of its plans'
// descriptions); an entry gives the value of one knob (PC_TUNE_*) at one
// transform length.
// ---------------------------------------------------------------------------
struct TuneEntry {
  uint64_t key;
  int knob, length, value;
};
void tune_set(const std::vector<TuneEntry>& entries);
// the entry's value, or `rule` when the table has none for (key, knob, length)
int tune_get(uint64_t key, int knob, int length, int rule);
// Whether the forward column kernel of length L1 runs its late-spectrum
// variant (spectrum loaded after the transform: fewer registers, no latency
// hiding), for a launch whose instances loop over several terms or have one
// term each: decided once per length and kind from the runtime's occupancy
// figures for both variants (the rule a tuning entry can override).
bool cols_fwd_late(int L1, bool multi_term);
// Whether the adjoint column kernel of length L1 loads the next spectrum
// column while it transforms the current one: decided once per length, true
// where the runtime's occupancy figures show it costs no resident workgroup;
// (the rule a tuning entry can override).
bool cols_adj_prefetch(int L1);
// Whether the row-inverse kernel of length L2 (small: the small-tile variant)
// loads the next plane's tile while it transforms the current one: decided
// once per variant, true where the runtime's figures show at least two waves
// per SIMD and no spilled registers (the rule a tuning entry can override).
bool rows_inv_pipe(int L2, bool small);
// Row kernels take 2 G rows per workgroup; the small-tile variant (fewer
// rows, more workgroups) serves single images too small to fill the chip.
int row_block_rows(int L2, bool small = false);
int col_block_cols(int L1);
int row_threads(int L2, bool small = false);
int col_threads(int L1);
// rows: the leading rows of each image the blocks cover (0: all N1; rounded
// up to whole row blocks); block_rows: rows per block (0: the tile of
// row_block_rows(L2, small))
void append_row_blocks(std::vector<BlockRef>& out, int job, int64_t n_img, int N1, int L2, int nq,
                       bool small = false, int rows = 0, int block_rows = 0);
void append_col_blocks(std::vector<BlockRef>& out, int job, int64_t n_img, int H2, int L1, int nsub);
const char* kernel_kind_name(int kind);
// img_limit: blocks of images >= img_limit return at once (their input and
// output need not exist)
LaunchStatus launch_set(const LaunchSet& ls, int64_t nblocks, const float* x_arg, float* y_arg, hipStream_t s,
                        Tracer* tr, int64_t img_limit = INT64_MAX);
// h (m x N1 x N2, lag layout) -> Hs, through the plan's spectra launch sets
LaunchStatus launch_spec2d(const Plan2D& p, const float* h, hipStream_t s);
// keep: store U_k into p.keep on the way (when the plan holds it)
LaunchStatus launch_fwd2d(const Plan2D& p, const float* u, float* y, int64_t batch, hipStream_t s,
                          Tracer* tr = nullptr, bool keep = false);
LaunchStatus launch_adj2d_tail(const Plan2D& p, float* x, int64_t batch, hipStream_t s, Tracer* tr = nullptr);
LaunchStatus launch_adj2d(const Plan2D& p, const float* v, float* x, int64_t batch, hipStream_t s,
                          Tracer* tr = nullptr);

// Table-driven transposes between planes of the internal column-major
// layout [f2][f1] (plan-owned) and the natural real-FFT layout [f1][f2]
// (f2 < H2 contiguous) at offsets of a caller's buffer, one job per plane;
// scale_mode 1 (export only): entries multiplied by c_f2 inv_n (c = 1 on the
// first and last column, 2 elsewhere), for gradients.
struct TransposeJob {
  float2* internal;
  int64_t ext_off;   // complex entries before the plane in the caller's buffer
  int N1, H2;
  int scale_mode;
  float inv_n;
  int64_t block0;    // first workgroup of the job in the launch
};
struct TransposeSet {
  const TransposeJob* jobs = nullptr;  // device
  int njobs = 0;
  int64_t blocks = 0;
};
// workgroups of one plane
int64_t transpose_blocks(int N1, int H2);
// to_internal: ext -> the jobs' planes; else the planes -> ext
LaunchStatus launch_transpose_set(const TransposeSet& ts, float2* ext, bool to_internal, hipStream_t s);

// Spectra as parameters (natural real-FFT layout) and their gradients.
LaunchStatus launch_spectra1d(const Small1D* ps, const Large1D* pl, const float2* in, float2* out, bool import,
                              hipStream_t s);
LaunchStatus launch_grad1d_small(const Small1D& p, const float* u, const float* gy, float2* gspec, int64_t batch,
                                 float2* work, hipStream_t s, Tracer* tr = nullptr);
LaunchStatus launch_grad1d_large(const Large1D& p, const float* u, const float* gy, float2* gspec, int64_t batch,
                                 float2* E, hipStream_t s, Tracer* tr = nullptr);
LaunchStatus launch_spectra2d(const Plan2D& p, const float2* in, float2* out, bool import, hipStream_t s);
// rows_u: transform b_q . u first (false: RA already holds them); keep:
// U_k kept by a forward pass (m x batch_cap planes), read instead of
// recomputed.  Leaves Tws = colFFT(rowFFT(gy)) and RA unchanged.
LaunchStatus launch_grad2d(const Plan2D& p, const float* u, const float* gy, float2* gspec, int64_t batch,
                           float2* E, hipStream_t s, Tracer* tr = nullptr, bool rows_u = true,
                           const float2* keep = nullptr);

// --------------------------------------------------------------------------
// 2D sectioned evaluation (compact supports; the complexity lemma of section
// 3.5, Lemma 3.2).  Term k only touches the p-sample box of its window and
// produces a (p + q - 1)-sample box of output (q: the box of h_k), so it is
// evaluated on its own M1 x M2 section (M >= p + q - 1 per axis, or M = N)
// by a single-term sub-operator, and the sections are added back.
// --------------------------------------------------------------------------
struct SecTerm {
  int64_t off;        // staging offset (floats) of the term's block: cap x M1 x M2
  int M1, M2;         // section size
  int gf1, gf2;       // forward: input box origin (the window box)
  int ga1, ga2;       // adjoint: input box origin (the output box)
  int sf1, sf2;       // forward: output box origin
  int ef1, ef2;       // forward: output box extent (p + q - 1, at most M)
  int sa1, sa2;       // adjoint: output box origin (the window box)
  int ea1, ea2;       // adjoint: output box extent (p)
};
struct Sec2D {
  int N1, N2, n_sec;
  int64_t cap;
  const SecTerm* terms;       // n_sec entries (device)
  float* Sout;                // section outputs (staging)
  // output tiles of SEC_TILE_R x SEC_TILE_C pixels: sections whose output
  // box meets each tile (CSR, section order), forward and adjoint
  int tiles2;
  const int* tf_off;
  const int* tf_items;
  const int* ta_off;
  const int* ta_items;
  // the window boxes partition the image: the adjoint's row-inverse pass
  // writes the output itself (no staging, no overlap-add)
  bool direct_adj = false;
};
constexpr int SEC_TILE_R = 32, SEC_TILE_C = 32;  // tile sides divide every supported size (>= 64, 2^a or 3 x 2^a)
// every output pixel of the first `batch` images <- sum of the sections
// covering it; the output is y, or (yp non-null) the pointer held at *yp
// when the kernel runs (a batch's table entry)
LaunchStatus launch_sec_scatter(const Sec2D& q, float* y, bool adjoint, int64_t batch, hipStream_t s, Tracer* tr,
                                float* const* yp = nullptr);

// --------------------------------------------------------------------------
// Construction of h_k from a TVIR (section 4.2 projection, section 4.4
// interpolation)
// --------------------------------------------------------------------------
constexpr int GEMM_WAVE_ROWS = 64, GEMM_ROWS = 4 * GEMM_WAVE_ROWS, GEMM_COLS = 32, GEMM_CHUNK = 2048;
constexpr int CONSTRUCT_MAX_M = 128;
inline int gemm_splits(int64_t K) { return (int)((K + GEMM_CHUNK - 1) / GEMM_CHUNK); }
// part[split][r][c] = sum over the split's chunk of A[r][j] B[c][j] (FP32 MFMA);
// K % 16 == 0, rows of A and B 16-byte aligned
LaunchStatus launch_gemm_nt(const float* A, int64_t rows, const float* B, int cols, int64_t K, float* part,
                            hipStream_t s);
LaunchStatus launch_sum_splits(const float* part, int splits, int64_t n, double* out, hipStream_t s);
LaunchStatus launch_cholesky(double* G, int m, int* fail, hipStream_t s);
LaunchStatus launch_lu(double* E, int m, int* perm, int* fail, hipStream_t s);
LaunchStatus launch_row_solve(bool lu, const double* F, const int* perm, int m, const double* src, double* work,
                              int64_t rows, const int64_t* lags, int64_t n, float* h, hipStream_t s);
LaunchStatus launch_fill_zero(float* x, int64_t n, hipStream_t s);
LaunchStatus launch_node_matrix(const float* W, int m, int64_t n, const int64_t* nodes, double* E, hipStream_t s);
LaunchStatus launch_to_double(const float* x, int64_t n, double* y, hipStream_t s);
LaunchStatus launch_flip(const float* in, float* out, int64_t count, int64_t n0, int64_t n1, hipStream_t s);

// --------------------------------------------------------------------------
// Periodic orthonormal wavelet transforms (section 4.5)
// --------------------------------------------------------------------------
constexpr int WAVELET_MAX_TAPS = 20;
struct WaveletFilter {
  int taps;
  float h[WAVELET_MAX_TAPS];  // lowpass
  float g[WAVELET_MAX_TAPS];  // highpass g[k] = (-1)^k h[taps - 1 - k]
};
// `levels` levels of the periodic DWT (synthesis: its inverse) of `count`
// vectors of n samples, element i of vector b at b * dist + i * stride (in
// and out alike); s1, s2: scratch of count * n / 2 floats each
LaunchStatus launch_wavelet(bool synthesis, int64_t n, int levels, const WaveletFilter& f, int64_t count,
                            int64_t stride, int64_t dist, const float* in, float* out, float* s1, float* s2,
                            hipStream_t s);
// The same transform with its two scratch buffers in a fixed device array
// of WAVELET_STATIC_FLOATS floats per device (no allocation): needs
// count * (n / 2) <= WAVELET_STATIC_FLOATS / 2 (hipErrorInvalidValue
// otherwise, nothing launched).  Calls that overlap on one device race.
constexpr int64_t WAVELET_STATIC_FLOATS = (int64_t)1 << 22;  // 16 MiB per device
LaunchStatus launch_wavelet_static(bool synthesis, int64_t n, int levels, const WaveletFilter& f, int64_t count,
                                   int64_t stride, int64_t dist, const float* in, float* out, hipStream_t s);

}  // namespace pc
