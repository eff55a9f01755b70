// Workgroup FFT engine for gfx950 (CDNA4, wave64).
//
// One L-point complex FFT is carried by T = L/P threads; thread t holds the
// P points x[t + T*e], e = 0..P-1, in registers, both before and after the
// transform (natural order, stride T).  The transform is a Stockham
// autosort sequence of radix-R passes (R divides P); between passes the data
// go through LDS (or, before a last radix-2 pass of a half-wavefront
// transform, across lanes: see XlTab), the last pass writes straight back to
// registers.  Because
// input and output live at the same register slots, the spectral
// multiply-accumulate and the inverse transform can follow the forward
// transform without any reordering.
//
// Sign convention (Fourier atoms of the notation section): forward
// X[f] = sum_n x[n] exp(-2 i pi f n / L); inverse is unnormalised with the
// opposite sign.
//
// Twiddles come from a per-(L, P) table built on the host in float64 and
// rounded once: for every pass (stride Ns, radix R) it lists
// exp(-2 i pi q k / (Ns R)) for k < Ns, 1 <= q < R, so one butterfly reads
// R-1 consecutive entries.  The table has L-1 entries.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pc {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
// acc + a*b
__device__ __forceinline__ float2 cfma(float2 acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
  return acc;
}
// acc + conj(a)*b
__device__ __forceinline__ float2 cfma_conj(float2 acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(-a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// small DFTs in registers
// ---------------------------------------------------------------------------
template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2* x) {
  const float c = -0.5f;
  const float s = INV ? 0.86602540378443864676f : -0.86602540378443864676f;
  float2 t = cadd(x[1], x[2]);
  float2 d = csub(x[1], x[2]);
  float2 m = make_float2(fmaf(c, t.x, x[0].x), fmaf(c, t.y, x[0].y));
  // i*s*d
  float2 r = make_float2(-s * d.y, s * d.x);
  x[0] = cadd(x[0], t);
  x[1] = cadd(m, r);
  x[2] = csub(m, r);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  float2 a = cadd(x0, x2), b = csub(x0, x2);
  float2 c = cadd(x1, x3), d = mul_mi<INV>(csub(x1, x3));
  x0 = cadd(a, c);
  x2 = csub(a, c);
  x1 = cadd(b, d);
  x3 = csub(b, d);
}

// W8^k for k = 1..3, forward sign exp(-2 i pi k/8)
template <bool INV>
__device__ __forceinline__ float2 w8_1(float2 a) {
  const float h = 0.70710678118654752440f;
  // forward: a * (1 - i)/sqrt2 ; inverse: a * (1 + i)/sqrt2
  return INV ? make_float2(h * (a.x - a.y), h * (a.x + a.y)) : make_float2(h * (a.x + a.y), h * (a.y - a.x));
}
template <bool INV>
__device__ __forceinline__ float2 w8_3(float2 a) {
  const float h = 0.70710678118654752440f;
  // forward: a * (-1 - i)/sqrt2 ; inverse: a * (-1 + i)/sqrt2
  return INV ? make_float2(-h * (a.x + a.y), h * (a.x - a.y)) : make_float2(h * (a.y - a.x), -h * (a.x + a.y));
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* x) {
  // even / odd 4-point transforms, then one radix-2 combine
  float2 e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  float2 o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  o1 = w8_1<INV>(o1);
  o2 = mul_mi<INV>(o2);
  o3 = w8_3<INV>(o3);
  x[0] = cadd(e0, o0); x[4] = csub(e0, o0);
  x[1] = cadd(e1, o1); x[5] = csub(e1, o1);
  x[2] = cadd(e2, o2); x[6] = csub(e2, o2);
  x[3] = cadd(e3, o3); x[7] = csub(e3, o3);
}

template <bool INV>
__device__ __forceinline__ void dft16(float2* x) {
  // 16 = 4 x 4: transforms over n2 of x[n1 + 4 n2], twiddle W16^(n1 k2),
  // transforms over n1; output index k2 + 4 k1.
  float2 a[16];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    float2 y0 = x[n1], y1 = x[n1 + 4], y2 = x[n1 + 8], y3 = x[n1 + 12];
    dft4<INV>(y0, y1, y2, y3);
    a[n1 * 4 + 0] = y0; a[n1 * 4 + 1] = y1; a[n1 * 4 + 2] = y2; a[n1 * 4 + 3] = y3;
  }
  // twiddles W16^(n1*k2): n1 in 1..3, k2 in 1..3
  const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
  const float h = 0.70710678118654752440f;
  const float sg = INV ? 1.0f : -1.0f;
  // W16^1, W16^2, W16^3, W16^4 = -i(fwd), W16^6, W16^9
  const float2 w1 = make_float2(c1, sg * s1);
  const float2 w2 = make_float2(h, sg * h);
  const float2 w3 = make_float2(s1, sg * c1);
  const float2 w6 = make_float2(-h, sg * h);
  const float2 w9 = make_float2(-c1, -sg * s1);
  a[1 * 4 + 1] = cmul(a[1 * 4 + 1], w1);
  a[1 * 4 + 2] = cmul(a[1 * 4 + 2], w2);
  a[1 * 4 + 3] = cmul(a[1 * 4 + 3], w3);
  a[2 * 4 + 1] = cmul(a[2 * 4 + 1], w2);
  a[2 * 4 + 2] = mul_mi<INV>(a[2 * 4 + 2]);
  a[2 * 4 + 3] = cmul(a[2 * 4 + 3], w6);
  a[3 * 4 + 1] = cmul(a[3 * 4 + 1], w3);
  a[3 * 4 + 2] = cmul(a[3 * 4 + 2], w6);
  a[3 * 4 + 3] = cmul(a[3 * 4 + 3], w9);
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    float2 y0 = a[0 * 4 + k2], y1 = a[1 * 4 + k2], y2 = a[2 * 4 + k2], y3 = a[3 * 4 + k2];
    dft4<INV>(y0, y1, y2, y3);
    x[k2 + 0] = y0; x[k2 + 4] = y1; x[k2 + 8] = y2; x[k2 + 12] = y3;
  }
}

// 12 points as a prime-factor 3 x 4 transform (no twiddles between the two
// stages): input n = (4 n1 + 3 n2) mod 12, output k = (4 k1 + 9 k2) mod 12,
// so that nk = 4 n1 k1 + 3 n2 k2 (mod 12): three-point transforms over n1,
// then four-point transforms over n2.
template <bool INV>
__device__ __forceinline__ void dft12(float2* x) {
  float2 a[3][4];
#pragma unroll
  for (int n1 = 0; n1 < 3; ++n1)
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) a[n1][n2] = x[(4 * n1 + 3 * n2) % 12];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    float2 t[3] = {a[0][n2], a[1][n2], a[2][n2]};
    dft3<INV>(t);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) a[k1][n2] = t[k1];
  }
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) dft4<INV>(a[k1][0], a[k1][1], a[k1][2], a[k1][3]);
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) x[(4 * k1 + 9 * k2) % 12] = a[k1][k2];
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(float2* x) {
  if constexpr (R == 2) dft2<INV>(x[0], x[1]);
  else if constexpr (R == 3) dft3<INV>(x);
  else if constexpr (R == 4) dft4<INV>(x[0], x[1], x[2], x[3]);
  else if constexpr (R == 8) dft8<INV>(x);
  else if constexpr (R == 16) dft16<INV>(x);
  else if constexpr (R == 12) dft12<INV>(x);
  else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// pass schedule
// ---------------------------------------------------------------------------
struct Sched {
  int n;
  int r[12];
};

// A radix-3 pass for L = 3 * 2^a (radix 12, the three-point and a
// four-point stage in one pass, at 12 points per thread), and passes of
// the largest power of two dividing P (capped at 16) with a smaller one if
// needed.
constexpr Sched make_sched(int L, int P) {
  Sched s{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
  int rem = L;
  if (rem % 12 == 0 && P == 12) {
    s.r[s.n++] = 12;
    rem /= 12;
  } else if (rem % 3 == 0) {
    s.r[s.n++] = 3;
    rem /= 3;
  }
  int p2 = P & -P;
  if (p2 > 16) p2 = 16;
  while (rem > 1) {
    int r = p2 < rem ? p2 : rem;
    s.r[s.n++] = r;
    rem /= r;
  }
  // the radix-12 pass second: a first pass writes its outputs at a stride
  // of R entries, which the pad period keeps free of bank conflicts for the
  // power-of-two radices but not for 12, and after a radix-4 first pass
  // its writes (runs of 4 entries, 48 apart) spread over the banks better
  // than a second radix-4 pass's (runs of 4, 16 apart)
  if (s.r[0] == 12 && s.n > 1) {
    s.r[0] = s.r[1];
    s.r[1] = 12;
  }
  return s;
}

constexpr bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

constexpr bool sched_ok(int L, int P) {
  if (L % P) return false;
  int rem = L;
  if (rem % 3 == 0) {
    rem /= 3;
    if (P % 3) return false;
  }
  if (!is_pow2(rem)) return false;
  Sched s = make_sched(L, P);
  for (int i = 0; i < s.n; ++i)
    if (P % s.r[i]) return false;
  return true;
}

// LDS word (float2) index with one pad slot per PAD entries: keeps the
// stride-R writes of the first passes free of bank conflicts.
// The default period suits the 2D kernels; the four-step 1D kernels use 32
// (fewer bank conflicts in their 512-thread exchanges, measured).
#ifndef PC_LDS_PAD
#define PC_LDS_PAD 16
#endif
constexpr int PAD = PC_LDS_PAD;
static_assert(PAD == 16 || PAD == 32, "pad period 16 or 32");
template <int PW = PAD>
__device__ __forceinline__ int lpad(int i) {
  // i >= 0: unsigned division by the power of two PW is one shift (a signed
  // one needs a sign fix-up)
  return i + (int)((unsigned)i / PW);
}
// The exchange after a radix-12 pass of stride Ns = 4 (the second pass at
// 12 points per thread) writes runs of 4 entries, 48 apart.  Under the pad
// above, the runs of one 16-lane pass overlap in the banks (two-way
// conflicts on every write).  That exchange instead skews by SKEW entries
// per block of SKEW_BLOCK: the runs start 4 entries (8 banks) apart, and a
// 16-aligned read of 16 consecutive entries stays in one block.
constexpr int SKEW_BLOCK = 48, SKEW = 4;
constexpr bool skew_reads_ok(int T, int P) {
  for (int e = 0; e < P; ++e)
    if ((T * e) % SKEW_BLOCK + T - 1 >= 2 * SKEW_BLOCK) return false;
  return true;
}

// Entries of one transform's LDS buffer: the padded layout, or the skewed
// one where it is longer (lengths at 12 points per thread).
template <int L, int PW = PAD>
constexpr int lds_len() {
  constexpr int pad = L + L / PW, skew = L + SKEW * ((L - 1) / SKEW_BLOCK);
  return (L % SKEW_BLOCK == 0 && L < 1536 && skew > pad) ? skew : pad;
}

// ---------------------------------------------------------------------------
// Synchronisation of the LDS exchanges.  A transform carried by T threads
// with T dividing the wavefront size (64) lives inside one wavefront, whose
// LDS operations the hardware performs in program order: its exchanges then
// need only a compiler-level barrier, not a workgroup barrier, and the other
// wavefronts of the workgroup run on.  SYNC_WG: every exchange waits on the
// workgroup (always correct); SYNC_WAVE_ENTRY: wave-local exchanges, but the
// first write still waits on the workgroup (the caller's LDS region was read
// by other wavefronts just before the transform); SYNC_WAVE: wave-local
// throughout (the region was last used by this transform's own threads).
// The wave-local modes fall back to SYNC_WG when T does not divide 64.
// ---------------------------------------------------------------------------
enum { SYNC_WG = 0, SYNC_WAVE_ENTRY = 1, SYNC_WAVE = 2 };

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int T, int SYNC>
constexpr int eff_sync() {
  return (T <= 64 && 64 % T == 0) ? SYNC : SYNC_WG;
}

template <int SYNC, bool ENTRY>
__device__ __forceinline__ void exchange_sync() {
  if constexpr (SYNC == SYNC_WG || (ENTRY && SYNC == SYNC_WAVE_ENTRY))
    __syncthreads();
  else
    wave_sync();
}

// ---------------------------------------------------------------------------
// Cross-lane exchange (a wavefront shuffle instead of an LDS round trip).
// Take a transform carried by T = 32 threads, one T-aligned half of a
// wavefront, whose last pass has radix 2, and the exchange that feeds that
// pass.  Every output of the pass before it then either stays in its thread
// or goes to the partner thread t xor 16.  Within each 16-lane half, one
// register of the same index feeds each destination register.  The
// exchange is then a register network: v_permlane16_swap (gfx950) swaps the
// odd 16-lane rows of its first operand with the even rows of its second.
// Lane t < 16 of the result's second register then holds the first
// operand's lane t + 16, and lane t >= 16 of the result's first register
// holds the second operand's lane t - 16.  So one swap per float component
// gives every lower lane one register of its upper partner and every upper
// lane one register of its lower partner.  make_xltab derives the network
// from the Stockham index map and checks it by emulating it; no LDS, no
// synchronisation.
// ---------------------------------------------------------------------------
struct XlTab {
  bool ok;
  int nsw;                  // swaps per float component
  int sx1[16], sx2[16];     // swap s: first operand o[sx1[s]], second o[sx2[s]]
  int lo[16], hi[16];       // destination e, lower / upper lanes: own o[x] (x >= 0) or swap -1 - x's result
};

template <int L, int P>
constexpr XlTab make_xltab() {
  XlTab x{};
  x.ok = false;
  constexpr int T = L / P;
  const Sched s = make_sched(L, P);
  if (T != 32 || P > 16 || s.n < 3 || s.r[s.n - 1] != 2) return x;
  int Ns = 1;
  for (int i = 0; i < s.n - 2; ++i) Ns *= s.r[i];
  const int R = s.r[s.n - 2], B = P / R;
  // destination (lane, register) <- source (lane, register) of the Stockham exchange
  int sl[32][16] = {}, sr[32][16] = {};
  for (int t = 0; t < T; ++t)
    for (int b = 0; b < B; ++b)
      for (int q = 0; q < R; ++q) {
        const int j = t + T * b, k = j % Ns, pos = (j / Ns) * Ns * R + k + q * Ns;
        sl[pos % T][pos / T] = t;
        sr[pos % T][pos / T] = b + q * B;
      }
  int lo_src[16] = {}, hi_src[16] = {}, nlo = 0, nhi = 0;
  for (int e = 0; e < P; ++e)
    for (int h = 0; h < 2; ++h) {
      const int t0 = 16 * h, d = sl[t0][e] ^ t0, r = sr[t0][e];
      if (d != 0 && d != 16) return x;
      for (int t = t0; t < t0 + 16; ++t)
        if ((sl[t][e] ^ t) != d || sr[t][e] != r) return x;
      if (h == 0) {
        x.lo[e] = d == 0 ? r : -1 - nlo;
        if (d != 0) lo_src[nlo++] = r;
      } else {
        x.hi[e] = d == 0 ? r : -1 - nhi;
        if (d != 0) hi_src[nhi++] = r;
      }
    }
  x.nsw = nlo > nhi ? nlo : nhi;
  for (int i = 0; i < x.nsw; ++i) {
    x.sx1[i] = i < nlo ? lo_src[i] : 0;
    x.sx2[i] = i < nhi ? hi_src[i] : 0;
  }
  // emulate the network: lane t < 16 reads swap i's second result, which
  // there is the first operand of lane t + 16; lane t >= 16 reads the first
  // result, there the second operand of lane t - 16
  for (int t = 0; t < T; ++t)
    for (int e = 0; e < P; ++e) {
      const bool lower = t < 16;
      const int c = lower ? x.lo[e] : x.hi[e];
      const int lane = c >= 0 ? t : (lower ? t + 16 : t - 16);
      const int reg = c >= 0 ? c : (lower ? x.sx1[-1 - c] : x.sx2[-1 - c]);
      if (lane != sl[t][e] || reg != sr[t][e]) return x;
    }
  x.ok = true;
  return x;
}

template <int L, int P>
struct Xl {
  static constexpr XlTab tab = make_xltab<L, P>();
};
static_assert(make_xltab<384, 12>().ok && make_xltab<512, 16>().ok, "cross-lane exchange of the 384- and 512-point transforms");

__device__ __forceinline__ float2 permlane16_swap_lower_upper(float2 a, float2 b, bool lower) {
  const auto sx = __builtin_amdgcn_permlane16_swap(__float_as_uint(a.x), __float_as_uint(b.x), false, false);
  const auto sy = __builtin_amdgcn_permlane16_swap(__float_as_uint(a.y), __float_as_uint(b.y), false, false);
  return lower ? make_float2(__uint_as_float(sx[1]), __uint_as_float(sy[1]))
               : make_float2(__uint_as_float(sx[0]), __uint_as_float(sy[0]));
}

// ---------------------------------------------------------------------------
// the engine
// ---------------------------------------------------------------------------
template <int L, int P, bool INV, int S, int Ns, int TW, int PW, int SYNC = SYNC_WG, bool XL = false>
struct FftPass {
  static constexpr Sched sch = make_sched(L, P);
  static constexpr int R = sch.r[S];
  static constexpr int B = P / R;
  static constexpr int T = L / P;
  static constexpr bool LAST = (S == sch.n - 1);
  // this pass feeds the last one across lanes
  static constexpr bool XLANE = XL && S == sch.n - 2 && Xl<L, P>::tab.ok;
  // this pass's exchange uses the skewed layout (see SKEW_BLOCK)
  static constexpr bool SKW = !LAST && !XLANE && R == 12 && Ns == 4;
  static_assert(!SKW || L + SKEW * ((L - 1) / SKEW_BLOCK) <= lds_len<L, PW>(), "LDS room for the skewed exchange");
  static_assert(!SKW || skew_reads_ok(T, P), "a skewed read of t + T e crosses one block boundary at most");

  __device__ __forceinline__ static void run(float2 (&v)[P], float2* lds, const float2* __restrict__ tw, int t) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      // unsigned: j / Ns and j % Ns by constants without sign fix-ups
      const unsigned j = (unsigned)t + T * b;
      const int k = (int)(j % Ns);
      float2 x[R];
#pragma unroll
      for (int q = 0; q < R; ++q) x[q] = v[b + q * B];
      if constexpr (Ns > 1) {
        const float2* w = tw + TW + k * (R - 1);
#pragma unroll
        for (int q = 1; q < R; ++q) {
          float2 ww = w[q - 1];
          if (INV) ww.y = -ww.y;
          x[q] = cmul(x[q], ww);
        }
      }
      dftR<R, INV>(x);
      if constexpr (LAST || XLANE) {
#pragma unroll
        for (int q = 0; q < R; ++q) v[b + q * B] = x[q];
      } else {
        if (b == 0) exchange_sync<SYNC, S == 0>();  // previous readers of this LDS region are done
        const int base = (int)(j / Ns) * Ns * R + k;
        // The padded index is base + constant whenever the R outputs stay
        // inside one PW-entry row (Ns R divides PW; base is then a multiple
        // of Ns R plus k < Ns) or step by whole rows (Ns a multiple of PW).
        if constexpr (SKW) {
          // the R outputs stay in block j / Ns of Ns R = SKEW_BLOCK entries
          float2* dst = lds + base + SKEW * (int)(j / Ns);
#pragma unroll
          for (int q = 0; q < R; ++q) dst[q * Ns] = x[q];
        } else if constexpr (Ns % PW == 0) {
          float2* dst = lds + lpad<PW>(base);
#pragma unroll
          for (int q = 0; q < R; ++q) dst[q * (Ns + Ns / PW)] = x[q];
        } else if constexpr (PW % (Ns * R) == 0) {
          float2* dst = lds + lpad<PW>(base);
#pragma unroll
          for (int q = 0; q < R; ++q) dst[q * Ns] = x[q];
        } else {
#pragma unroll
          for (int q = 0; q < R; ++q) lds[lpad<PW>(base + q * Ns)] = x[q];
        }
      }
    }
    if constexpr (XLANE) {
      // the outputs sit at v[b + q B]; route them to the next pass's layout
      constexpr XlTab X = Xl<L, P>::tab;
      const bool lower = (t & 16) == 0;
      float2 o[P], rcv[X.nsw > 0 ? X.nsw : 1];
#pragma unroll
      for (int e = 0; e < P; ++e) o[e] = v[e];
#pragma unroll
      for (int i = 0; i < X.nsw; ++i) rcv[i] = permlane16_swap_lower_upper(o[X.sx1[i]], o[X.sx2[i]], lower);
#pragma unroll
      for (int e = 0; e < P; ++e) {
        const float2 a = X.lo[e] >= 0 ? o[X.lo[e] >= 0 ? X.lo[e] : 0] : rcv[X.lo[e] < 0 ? -1 - X.lo[e] : 0];
        const float2 c = X.hi[e] >= 0 ? o[X.hi[e] >= 0 ? X.hi[e] : 0] : rcv[X.hi[e] < 0 ? -1 - X.hi[e] : 0];
        v[e] = lower ? a : c;
      }
      FftPass<L, P, INV, S + 1, Ns * R, TW + Ns * (R - 1), PW, SYNC, XL>::run(v, lds, tw, t);
    } else if constexpr (!LAST) {
      exchange_sync<SYNC, false>();
      if constexpr (SKW) {
        // lskew(t + T e) = t + T e + SKEW (T e / SKEW_BLOCK) + SKEW [t + T e mod SKEW_BLOCK >= SKEW_BLOCK]
#pragma unroll
        for (int e = 0; e < P; ++e) {
          const int m = (T * e) % SKEW_BLOCK;
          v[e] = lds[t + T * e + SKEW * ((T * e) / SKEW_BLOCK) + (t + m >= SKEW_BLOCK ? SKEW : 0)];
        }
      } else if constexpr (T % PW == 0) {
        // (t + T e) / PW = t / PW + e T / PW
        const float2* src = lds + lpad<PW>(t);
#pragma unroll
        for (int e = 0; e < P; ++e) v[e] = src[e * (T + T / PW)];
      } else {
#pragma unroll
        for (int e = 0; e < P; ++e) v[e] = lds[lpad<PW>(t + T * e)];
      }
      FftPass<L, P, INV, S + 1, Ns * R, TW + Ns * (R - 1), PW, SYNC, XL>::run(v, lds, tw, t);
    }
  }
};

// ---------------------------------------------------------------------------
// Register-resident twiddles.  Every thread's twiddles depend only on its
// index, so a kernel that runs many transforms of the same length can load
// them once (tw_reg_count values per thread) and keep them in registers; the
// passes then read no twiddles from memory.  Same passes, same order, same
// values as fft_wg.
// ---------------------------------------------------------------------------
template <int L, int P>
constexpr int tw_reg_count() {
  Sched s = make_sched(L, P);
  int n = 0, Ns = 1;
  for (int i = 0; i < s.n; ++i) {
    if (Ns > 1) n += (P / s.r[i]) * (s.r[i] - 1);
    Ns *= s.r[i];
  }
  return n;
}

template <int L, int P, int S, int Ns, int TW, int RO>
struct TwRegLoad {
  static constexpr Sched sch = make_sched(L, P);
  static constexpr int R = sch.r[S];
  static constexpr int B = P / R;
  static constexpr int T = L / P;
  __device__ __forceinline__ static void run(float2* twr, const float2* __restrict__ tw, int t) {
    if constexpr (Ns > 1) {
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int k = (t + T * b) % Ns;
#pragma unroll
        for (int q = 1; q < R; ++q) twr[RO + b * (R - 1) + q - 1] = tw[TW + k * (R - 1) + q - 1];
      }
    }
    if constexpr (S + 1 < sch.n)
      TwRegLoad<L, P, S + 1, Ns * R, TW + Ns * (R - 1), RO + (Ns > 1 ? B * (R - 1) : 0)>::run(twr, tw, t);
  }
};

template <int L, int P, int NT>
__device__ __forceinline__ void load_tw_reg(float2 (&twr)[NT], const float2* __restrict__ tw, int t) {
  static_assert(NT == tw_reg_count<L, P>(), "register twiddle count");
  TwRegLoad<L, P, 0, 1, 0, 0>::run(twr, tw, t);
}

template <int L, int P, bool INV, int S, int Ns, int RO, int PW, bool PP>
struct FftPassReg {
  static constexpr Sched sch = make_sched(L, P);
  static constexpr int R = sch.r[S];
  static constexpr int B = P / R;
  static constexpr int T = L / P;
  static constexpr bool LAST = (S == sch.n - 1);

  template <int NTW>
  __device__ __forceinline__ static void run(float2 (&v)[P], float2* lds0, float2* lds1, const float2 (&twr)[NTW],
                                             int t) {
    // exchange S goes through lds0 (S even) or lds1 (S odd, ping-pong only)
    // (signed index arithmetic here: the unsigned form of FftPass took the
    // 4096-point four-step forward kernel from 251 to 256 VGPRs, one wave
    // per SIMD instead of two)
    float2* lds = (PP && (S & 1)) ? lds1 : lds0;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + T * b;
      const int k = j % Ns;
      float2 x[R];
#pragma unroll
      for (int q = 0; q < R; ++q) x[q] = v[b + q * B];
      if constexpr (Ns > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          float2 ww = twr[RO + b * (R - 1) + q - 1];
          if (INV) ww.y = -ww.y;
          x[q] = cmul(x[q], ww);
        }
      }
      dftR<R, INV>(x);
      if constexpr (LAST) {
#pragma unroll
        for (int q = 0; q < R; ++q) v[b + q * B] = x[q];
      } else {
        // previous readers of this LDS region are done (ping-pong: they
        // read before the barrier that ended the previous exchange)
        if (b == 0 && !PP) __syncthreads();
        const int base = (j / Ns) * Ns * R + k;
        if constexpr (Ns % PW == 0) {
          float2* dst = lds + lpad<PW>(base);
#pragma unroll
          for (int q = 0; q < R; ++q) dst[q * (Ns + Ns / PW)] = x[q];
        } else if constexpr (PW % (Ns * R) == 0) {
          float2* dst = lds + lpad<PW>(base);
#pragma unroll
          for (int q = 0; q < R; ++q) dst[q * Ns] = x[q];
        } else {
#pragma unroll
          for (int q = 0; q < R; ++q) lds[lpad<PW>(base + q * Ns)] = x[q];
        }
      }
    }
    if constexpr (!LAST) {
      __syncthreads();
      if constexpr (T % PW == 0) {
        const float2* src = lds + lpad<PW>(t);
#pragma unroll
        for (int e = 0; e < P; ++e) v[e] = src[e * (T + T / PW)];
      } else {
#pragma unroll
        for (int e = 0; e < P; ++e) v[e] = lds[lpad<PW>(t + T * e)];
      }
      FftPassReg<L, P, INV, S + 1, Ns * R, RO + (Ns > 1 ? B * (R - 1) : 0), PW, PP>::run(v, lds0, lds1, twr, t);
    }
  }
};

template <int L, int P, bool INV, int PW = PAD, int NT>
__device__ __forceinline__ void fft_wg_reg(float2 (&v)[P], float2* lds, const float2 (&twr)[NT], int t) {
  static_assert(sched_ok(L, P), "unsupported (L, P)");
  static_assert(NT == tw_reg_count<L, P>(), "register twiddle count");
  FftPassReg<L, P, INV, 0, 1, 0, PW, false>::run(v, lds, lds, twr, t);
}

// LDS exchanges of one transform (passes - 1).
template <int L, int P>
constexpr int fft_exchanges() {
  return make_sched(L, P).n - 1;
}

// Ping-pong form: consecutive exchanges alternate between two LDS buffers,
// so a pass writes without first waiting for the readers of the exchange
// before: every thread read that one before it wrote the previous exchange,
// hence before the barrier that ended it.  The alternation must continue
// across calls: the caller swaps buf[0] and buf[1] after every call when
// fft_exchanges<L, P>() is odd.  Costs a second buffer of lds_len entries;
// pays where the workgroup is the only one on its compute unit.
template <int L, int P, bool INV, int PW, int NT>
__device__ __forceinline__ void fft_wg_reg_pp(float2 (&v)[P], float2* const (&buf)[2], const float2 (&twr)[NT],
                                              int t) {
  static_assert(sched_ok(L, P), "unsupported (L, P)");
  static_assert(NT == tw_reg_count<L, P>(), "register twiddle count");
  FftPassReg<L, P, INV, 0, 1, 0, PW, true>::run(v, buf[0], buf[1], twr, t);
}

// Copy an engine twiddle table (L entries) into LDS.  Every thread of the
// workgroup calls it; it ends with a barrier.  Reading twiddles from LDS
// keeps the per-pass global-memory round trips off the transform.
template <int L>
__device__ __forceinline__ void stage_twiddles(float2* tw_lds, const float2* __restrict__ tw) {
  for (int i = threadIdx.x; i < L; i += blockDim.x) tw_lds[i] = tw[i];
  __syncthreads();
}

// The same staging in two steps, for NT threads: load() issues the table's
// loads into registers, commit() stores them into LDS and ends with a
// barrier.  A kernel issues its own first loads in between, so that the
// twiddles' round trip overlaps them instead of preceding them.
template <int L, int NT>
struct TwStage {
  static constexpr int N = (L + NT - 1) / NT;
  float2 r[N];
  __device__ __forceinline__ void load(const float2* __restrict__ tw, int tid) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int idx = tid + i * NT;
      if (tid < NT && idx < L) r[i] = tw[idx];
    }
  }
  __device__ __forceinline__ void commit(float2* tw_lds, int tid) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int idx = tid + i * NT;
      if (tid < NT && idx < L) tw_lds[idx] = r[i];
    }
    __syncthreads();
  }
};

// In-place transform of the register array v (see the header comment).
// Every thread of the workgroup must call it (it contains barriers), even
// threads whose FFT slot is unused.
template <int L, int P, bool INV, int PW = PAD>
__device__ __forceinline__ void fft_wg(float2 (&v)[P], float2* lds, const float2* __restrict__ tw, int t) {
  static_assert(sched_ok(L, P), "unsupported (L, P)");
  FftPass<L, P, INV, 0, 1, 0, PW>::run(v, lds, tw, t);
}

// The same transform with the exchange synchronisation SYNC (see SYNC_WG):
// wave-local exchanges where the T = L/P threads of a transform share one
// wavefront, and the cross-lane exchange of XlTab where it applies.  Threads
// of one transform must be consecutive and T-aligned (transform slot
// c = threadIdx.x / T, t = threadIdx.x mod T), as in every caller.
template <int L, int P, bool INV, int SYNC, int PW = PAD>
__device__ __forceinline__ void fft_wv(float2 (&v)[P], float2* lds, const float2* __restrict__ tw, int t) {
  static_assert(sched_ok(L, P), "unsupported (L, P)");
  FftPass<L, P, INV, 0, 1, 0, PW, eff_sync<L / P, SYNC>(), true>::run(v, lds, tw, t);
}

}  // namespace pc
