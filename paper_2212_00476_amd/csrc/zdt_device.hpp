// zdt_device.hpp -- gfx950 kernels of the stereo hot path.
//
//   hpass_kernel   one workgroup per (row y, chunk of LPS disparities); lanes map
//                  to d, each group of LPS lanes owns one contiguous x-segment of
//                  the row (LPS = 64: one segment per wave; LPS = 32: two).
//                  Modes: the exact int32 cross sums, the ZNCC cost (Sec. III-A,
//                  Eq. OP_ZNCC), the cost fused with the L and R passes
//                  (Eqs. DT1-DT2), or the L and R passes over a stored volume.
//   vpass_kernel   one workgroup per (column x, chunk of 64*DPL disparities);
//                  lanes map to d, each wave owns one y-segment of the column.
//                  U and D passes (Eqs. DT3-DT4), optionally fused with the WTA
//                  of Eq. WTA1 so that the last volume is never written.
//   wta_kernel     standalone WTA over a stored volume; one wave per pixel.
//
// A line (a row for H, a column for V) is split into segments.  Every pass is a
// first-order linear recursion c[i] += w[i] * c[i-1], so a segment's result is
// its carry-free local result plus (product of its weights) x (carry in).  The
// carries are composed across the segments of the workgroup through LDS, then
// each segment re-runs its recursion from the true carry: the values written
// are the sequential recursion of the paper apart from the rounding of the
// carries.  A segment's values stay in registers between the passes, so each
// kernel reads and writes the volume once.
//
// Volume accesses use raw buffer instructions: one VGPR offset per lane and the
// per-step offset in an SGPR, every offset inside the buffer by construction, so
// no address is kept per value.  Per-step LDS reads use one base address plus
// immediate offsets: the LDS line arrays carry SEG entries of padding so steps
// past a short segment need no clamping (their results are discarded).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace zdt {

constexpr int kWave = 64;
constexpr int kMaxWaves = 16;
constexpr int kMaxSegs = 32;   // segments per H workgroup (LPS = 32: two per wave)
constexpr int kGainBias = 13;  // FP16 working volume: value = fp16 * 2^(floor(log2 G) - kGainBias)

struct bf16 {
  uint16_t bits;
};
// FP16 element of a working volume scaled per pixel by its DT gain (see
// "Narrow working volumes" below); stored like _Float16.
struct f16x {
  _Float16 h;
};

typedef __amdgpu_buffer_rsrc_t rsrc_t;

// Raw buffer over [base, base + bytes).  base and bytes are workgroup-uniform;
// passing them through readfirstlane lets the compiler keep the descriptor in
// SGPRs (otherwise every access is wrapped in a waterfall loop).
__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  const uint64_t b = (uint64_t)base;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  const int n = __builtin_amdgcn_readfirstlane((int)bytes);
  void* p = (void*)(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, n, 0x00020000);
}

template <typename T>
struct Elem;
template <>
struct Elem<float> {
  static __device__ __forceinline__ float load(const float* p) { return *p; }
  static __device__ __forceinline__ void store(float* p, float v) { *p = v; }
  static __device__ __forceinline__ uint32_t braw(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
  }
  static __device__ __forceinline__ float decode(uint32_t u) { return __uint_as_float(u); }
  static __device__ __forceinline__ float bload(rsrc_t r, uint32_t voff, uint32_t soff) {
    return decode(braw(r, voff, soff));
  }
  static __device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, 0);
  }
};
template <>
struct Elem<_Float16> {
  static __device__ __forceinline__ float load(const _Float16* p) { return (float)*p; }
  static __device__ __forceinline__ void store(_Float16* p, float v) { *p = (_Float16)v; }
  static __device__ __forceinline__ uint32_t braw(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
  }
  static __device__ __forceinline__ float decode(uint32_t u) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)u);
  }
  static __device__ __forceinline__ float bload(rsrc_t r, uint32_t voff, uint32_t soff) {
    return decode(braw(r, voff, soff));
  }
  static __device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)v), r, (int)voff, (int)soff,
                                          0);
  }
};
template <>
struct Elem<f16x> {
  static __device__ __forceinline__ uint32_t braw(rsrc_t r, uint32_t voff, uint32_t soff) {
    return Elem<_Float16>::braw(r, voff, soff);
  }
  static __device__ __forceinline__ float decode(uint32_t u) { return Elem<_Float16>::decode(u); }
  static __device__ __forceinline__ float bload(rsrc_t r, uint32_t voff, uint32_t soff) {
    return Elem<_Float16>::bload(r, voff, soff);
  }
  static __device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, float v) {
    Elem<_Float16>::bstore(r, voff, soff, v);
  }
};
template <>
struct Elem<bf16> {
  // round to nearest even: one v_cvt_pk_bf16_f32 on gfx950
  static __device__ __forceinline__ uint16_t encode(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
  static __device__ __forceinline__ float load(const bf16* p) { return __uint_as_float((uint32_t)p->bits << 16); }
  static __device__ __forceinline__ void store(bf16* p, float v) { p->bits = encode(v); }
  static __device__ __forceinline__ uint32_t braw(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
  }
  static __device__ __forceinline__ float decode(uint32_t u) { return __uint_as_float(u << 16); }
  static __device__ __forceinline__ float bload(rsrc_t r, uint32_t voff, uint32_t soff) {
    return decode(braw(r, voff, soff));
  }
  static __device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b16(encode(v), r, (int)voff, (int)soff, 0);
  }
};

// Integer cost volumes of Sec. IV-C: the cost scaled by T and rounded to a
// 16-bit integer (i16v), or that integer's 8-bit code (i8c).  The passes run
// on the T-scaled values, so a stored state is read back exactly.
struct i16v {
  int16_t v;
};
struct i8c {
  uint8_t c;
};
template <typename T>
constexpr bool is_int_vol() {
  return std::is_same<T, i16v>::value || std::is_same<T, i8c>::value;
}

// float -> int16 with round-to-nearest-even and saturation, as an integer and
// as the float it stores exactly.
__device__ __forceinline__ float rq16(float v) { return __builtin_amdgcn_fmed3f(rintf(v), -32768.0f, 32767.0f); }
__device__ __forceinline__ int sat16(float v) { return (int)rq16(v); }

// 8-bit code of a 16-bit value (Sec. IV-C): non-negative values give 0; a
// negative value keeps the six bits below its leading ones at bit 9, 5 or 1
// (it lies below -2048, in [-2048, -128) or in [-128, 0)) with flag 1, 2 or 3.
__device__ __forceinline__ uint32_t i8_encode(int v) {
  const int pos = v < -2048 ? 9 : (v < -128 ? 5 : 1);
  const uint32_t flag = v < -2048 ? 1u : (v < -128 ? 2u : 3u);
  const uint32_t code = ((((uint32_t)v >> pos) & 0x3Fu) << 2) | flag;
  return v < 0 ? code : 0u;
}
// Its inverse: the six bits back at their position, ones above, zeros below
// (0, and the never-produced flag 0, give 0).
__device__ __forceinline__ int i8_decode(uint32_t c) {
  const uint32_t flag = c & 3u;
  const int pos = flag == 1u ? 9 : (flag == 2u ? 5 : 1);
  const int v = (int)((0xFFFFFFFFu << (pos + 6)) | ((c >> 2) << pos));  // sign-extended
  return flag ? v : 0;
}

template <>
struct Elem<i16v> {
  static __device__ __forceinline__ float load(const i16v* p) { return (float)p->v; }
  static __device__ __forceinline__ uint32_t braw(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
  }
  static __device__ __forceinline__ float decode(uint32_t u) { return (float)(short)(unsigned short)u; }
  static __device__ __forceinline__ float bload(rsrc_t r, uint32_t voff, uint32_t soff) {
    return decode(braw(r, voff, soff));
  }
  static __device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)sat16(v), r, (int)voff, (int)soff, 0);
  }
  static __device__ __forceinline__ void store(i16v* p, float v) { p->v = (int16_t)sat16(v); }
};
template <>
struct Elem<i8c> {
  static __device__ __forceinline__ float load(const i8c* p) { return (float)i8_decode(p->c); }
  static __device__ __forceinline__ uint32_t braw(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b8(r, (int)voff, (int)soff, 0);
  }
  static __device__ __forceinline__ float decode(uint32_t u) { return (float)i8_decode(u & 0xFFu); }
  static __device__ __forceinline__ float bload(rsrc_t r, uint32_t voff, uint32_t soff) {
    return decode(braw(r, voff, soff));
  }
  static __device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b8((unsigned char)i8_encode(sat16(v)), r, (int)voff, (int)soff, 0);
  }
  static __device__ __forceinline__ void store(i8c* p, float v) { p->c = (uint8_t)i8_encode(sat16(v)); }
};

__host__ __device__ constexpr int packs_of(int R) { return (2 * R + 1 + 3) / 4; }

// Register discipline for the unrolled recursions.  Without it the compiler
// issues a whole line's LDS weight reads first and sinks the (arithmetic-only)
// recursion below them, keeping one VGPR per step live.  Every kBlock steps the
// running values are pinned in place and memory is fenced, so each block's
// reads are consumed before the next block's are issued.
constexpr int kBlock = 8;
template <typename V>
__device__ __forceinline__ void pin1(V& v) {
  asm volatile("" : "+v"(v));
}
template <typename... V>
__device__ __forceinline__ void pin(V&... v) {
  (pin1(v), ...);
}
__device__ __forceinline__ void fence() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}
template <typename... V>
__device__ __forceinline__ void step_fence(int k, V&... v) {
  if (k % kBlock == kBlock - 1) {
    pin(v...);
    fence();
  }
}
// Re-read LDS weights in each pass instead of keeping a line of them live.
__device__ __forceinline__ void reload_fence() { asm volatile("" ::: "memory"); }

// Exact value entering segment `seg` of a split first-order recursion.
// Segment s maps an incoming value c to A[s] * c + B[s * ncol + col] (its weight
// product and its carry-free end value); the carry is the composition, in
// recursion order, of the segments before `seg` (0..seg-1; REV: n-1 down to
// seg+1) applied to 0.  The loads of a block of kCarryBlock segments are issued
// together, so a block costs one LDS round trip instead of one per segment.
// `max_count` is a wave-uniform bound on the number of segments to compose.
constexpr int kCarryBlock = 4;
template <bool REV>
__device__ __forceinline__ float carry_in(const float* B, const float* A, int seg, int n, int ncol, int col,
                                          int max_count) {
  const int count = REV ? n - 1 - seg : seg;
  float carry = 0.0f;
  for (int t0 = 0; t0 < max_count; t0 += kCarryBlock) {
    float a[kCarryBlock], b[kCarryBlock];
#pragma unroll
    for (int i = 0; i < kCarryBlock; ++i) {
      const int t = min(t0 + i, n - 1);  // position in recursion order (clamped; unused past count)
      const int s = REV ? n - 1 - t : t;
      a[i] = A[s];
      b[i] = B[s * ncol + col];
    }
#pragma unroll
    for (int i = 0; i < kCarryBlock; ++i) carry = (t0 + i < count) ? fmaf(a[i], carry, b[i]) : carry;
  }
  return carry;
}

// ---------------------------------------------------------------------------
// LDS layout of hpass_kernel, in 32-bit words (P = LPS - 1); every line array
// below is followed by `pad` (= SEG) spare entries.
//   LR[W+2R][RS]  one record of RS = rec_words(R) words per entry i: the packed
//                 column bytes of the reference rows y-R..y+R at column
//                 clamp(i-R) (byte j of pack k is row y-R+4k+j, clamped, zero
//                 past row y+R), then, for entries i < W, -S_R(i) and
//                 1/sqrt(l^2 S_RR - S_R^2) (0 for zero variance) of position i.
//   TR[W+P+2R][RS] target records: entry i packs column clamp(i-P-R-d0) and,
//                 for i < W+P, holds S_T (not negated) and the inverse
//                 deviation at x' = i-P-d0.
//   A lane's cost at x0+k reads records at constant offsets from two per-lane
//   bases; the odd stride keeps lanes that read consecutive records on distinct
//   banks.
//   WH[W+1]       W_L(x) for x in [0, W]; WH[0] = WH[W] = 0.
//   EX, EX2 [16*64], EXS, EXS2 [kMaxSegs]   segment carries.
//   GI, GO [W]    gains of the row before and after the pass pair (FP16
//                 working volumes only); after the pair's gain line is done,
//                 GO holds the output scale factors 2^(kGainBias - e) instead.
//   SI [W]        input scale factors 2^(e - kGainBias) of the stored input
//                 (FP16 H pairs over a stored volume only).
// ---------------------------------------------------------------------------
struct HLayout {
  int nLP, nTP, nTS, oLP, oTP, oWH, oEX, oEXS, oEX2, oEXS2, oGI, oGO, oSI, words;
};

// Words per column record: the packs, the window sum and 1/sigma, rounded up to odd.
__host__ __device__ constexpr int rec_words(int R) { return (packs_of(R) + 2) | 1; }

__host__ __device__ constexpr HLayout h_layout(int W, int R, int LPS, int pad, bool zncc, bool dt, bool scaled) {
  HLayout L{};
  const int RS = rec_words(R);
  // records: a row's W + 2R (reference) or nTS + 2R (target) columns, then
  // padding (at least the kStatRun - 1 columns a statistics run reads past them)
  L.nLP = W + 2 * R + (pad > 4 ? pad : 4);
  L.nTS = W + LPS - 1;
  L.nTP = L.nTS + 2 * R + (pad > 4 ? pad : 4);
  int o = 0;
  if (zncc) {
    L.oLP = o; o += RS * L.nLP;
    L.oTP = o; o += RS * L.nTP;
  }
  if (dt) {
    L.oWH = o; o += W + 1 + pad;
    L.oEX = o; o += kMaxWaves * kWave;
    L.oEXS = o; o += kMaxSegs;
    L.oEX2 = o; o += kMaxWaves * kWave;
    L.oEXS2 = o; o += kMaxSegs;
    L.oGI = o;
    if (scaled) o += W + pad;  // FP16 working volume: the row's gains before and after the pair
    L.oGO = o;
    if (scaled) o += W + pad;
    L.oSI = o;
    if (scaled && !zncc) o += W + pad;
  }
  L.words = o;
  return L;
}

enum HMode { kSums = 0, kCost = 1, kCostHPair = 2, kHPair = 3 };

// The normalization of the integer volumes (Sec. IV-C, Eq. DT_new with
// d_arb = 0) follows the FastDT of Sec. V-C: in the U2D pass for Int16, in the
// R2L pass for Int8, subtracting the pass input's d = 0 value at each pixel.
// Only the first sweep needs it (the d = 0 slice is zero from then on).  That
// slice of the subtracted state lives in another workgroup (disparity chunk
// 0), so it goes through a [H][W] map:
//   kRefNone       no map
//   kRefL2ROut     Int8 reference launch (chunk 0 only): lane d = 0 writes its
//                  stored L2R output and the workgroup ends after the L pass
//   kRefL2RIn      Int8 fused pass: the map is subtracted from the stored L2R
//                  output before the R2L recursion
//   kRefR2LOut     Int16 fused pass: lane d = 0 also writes its stored R2L
//                  output to the map (the V pair of the first sweep subtracts it)
// The reference launch runs the same code as the fused pass up to the L
// output, so the subtracted values equal chunk 0's own bit for bit and the
// normalized d = 0 slice is exactly zero.
enum IntRef { kRefNone = 0, kRefL2ROut = 1, kRefL2RIn = 2, kRefR2LOut = 3 };

struct HArgs {
  const uint8_t* left;
  const uint8_t* right;
  const uint8_t* guide;
  int pitch, W, H, D;
  float inv_sigma_s, range_coef, out_scale;
  float cost_scale;      // integer volumes: T, applied to the raw cost of the fused pass
  int ref_role;          // integer volumes, first sweep: what `ref` is for (IntRef)
  float* ref;            // [H][W] d_arb = 0 slice of a stored state (see IntRef)
  void* vol;
  int32_t* s_rt;
  int32_t* s_l;
  int32_t* s_ll;
  int32_t* s_t;
  int32_t* s_tt;
  const float* g_in;  // FP16 working volume: gain map [H][W] of the stored input (sweeps 2..I)
  float* g_out;       // and of the output (written by the workgroups of chunk 0)
  int segl, nseg;     // segment length and number of segments of a row
  int nchunks;     // disparity chunks of LPS lanes per row
};

// Multi-job launches: grid z indexes the job, and each job's buffers come from
// a pointer table passed with the kernel arguments (jobs of one launch share
// shape and parameters; a single job is a table of one).
constexpr int kMaxJobs = 32;
struct HJob {
  const uint8_t* left;
  const uint8_t* right;
  const uint8_t* guide;
  void* vol;
  const float* g_in;
  float* g_out;
  float* ref;
};
struct HJobs {
  HJob j[kMaxJobs];
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// DT weight between G(a) and its predecessor G(b): exp(-1/sigma_s - |G(a)-G(b)| / (255 sigma_r)).
__device__ __forceinline__ float dt_weight(int ga, int gb, float inv_sigma_s, float range_coef) {
  return expf(-(inv_sigma_s + (float)abs(ga - gb) * range_coef));
}

// Window sums of one image at kStatRun consecutive positions: the column sums
// (of I and I^2, by dot4 over the packed rows) of the kStatRun + 2R columns
// involved are formed once and the window slides over them.  P holds column
// records (packs first); position p covers records p .. p+2R.
// Five positions per run: lanes then read records 5 * RS words apart, an odd
// stride, so a wave's reads fall on distinct banks.
constexpr int kStatRun = 5;
static_assert(kStatRun - 1 <= 4, "record padding of h_layout");
template <int R>
__device__ __forceinline__ void window_run(const uint32_t* P, int p0, uint32_t (&s)[kStatRun],
                                           uint32_t (&ss)[kStatRun]) {
  constexpr int NP = packs_of(R);
  constexpr int RS = rec_words(R);
  constexpr int NW = 2 * R + 1;
  constexpr int NC = kStatRun + 2 * R;
  uint32_t cs[NC], css[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const int col = p0 + j;  // up to kStatRun - 1 columns past the row: padding of the array
    cs[j] = 0;
    css[j] = 0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const uint32_t v = P[col * RS + k];
      cs[j] = __builtin_amdgcn_udot4(v, 0x01010101u, cs[j], false);
      css[j] = __builtin_amdgcn_udot4(v, v, css[j], false);
    }
  }
  uint32_t a = 0, b = 0;
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    a += cs[j];
    b += css[j];
  }
  s[0] = a;
  ss[0] = b;
#pragma unroll
  for (int i = 1; i < kStatRun; ++i) {
    a += cs[i + 2 * R] - cs[i - 1];
    b += css[i + 2 * R] - css[i - 1];
    s[i] = a;
    ss[i] = b;
  }
}

// Stage the packed window columns and the per-position window statistics of
// both images for row y and disparity chunk d0 (reads the 2R+1 image rows once).
template <int R, int LPS>
__device__ void stage_zncc(const HArgs& a, const HLayout& lay, uint32_t* smem, int y, int d0, int mode) {
  constexpr int NP = packs_of(R);
  constexpr int NW = 2 * R + 1;
  constexpr int N = NW * NW;
  constexpr int P = LPS - 1;
  constexpr int RS = rec_words(R);
  const int tid = threadIdx.x, nt = blockDim.x, W = a.W, H = a.H;
  uint32_t* LR = smem + lay.oLP;
  uint32_t* TR = smem + lay.oTP;
  const uint8_t* lrow[NW];
  const uint8_t* trow[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const size_t off = (size_t)clampi(y - R + q, 0, H - 1) * a.pitch;
    lrow[q] = a.left + off;
    trow[q] = a.right + off;
  }
  // pack j of a column holds rows 4j .. 4j+3 of the window, one byte each
  // (bytes past the window's last row are zero)
  for (int i = tid; i < W + 2 * R; i += nt) {
    const int col = clampi(i - R, 0, W - 1);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      uint32_t p = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (4 * k + j < NW) p |= (uint32_t)lrow[4 * k + j][col] << (8 * j);
      LR[i * RS + k] = p;
    }
  }
  for (int i = tid; i < lay.nTS + 2 * R; i += nt) {
    const int col = clampi(i - P - R - d0, 0, W - 1);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      uint32_t p = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (4 * k + j < NW) p |= (uint32_t)trow[4 * k + j][col] << (8 * j);
      TR[i * RS + k] = p;
    }
  }
  __syncthreads();
  // Runs of kStatRun positions: the first nrl threads take the reference
  // positions x (columns x-R..x+R are LR entries x .. x+2R), the next nrt the
  // target positions t, i.e. x' = t - P - d0 (TR entries t .. t+2R).  The
  // statistics go to words NP, NP+1 of a position's own record, which no run
  // reads.
  const int nrl = (W + kStatRun - 1) / kStatRun;
  const int nrt = (lay.nTS + kStatRun - 1) / kStatRun;
  for (int u = tid; u < nrl + nrt; u += nt) {
    const bool ref = u < nrl;
    const int p0 = (ref ? u : u - nrl) * kStatRun;
    uint32_t s[kStatRun], ss[kStatRun];
    window_run<R>(ref ? LR : TR, p0, s, ss);
#pragma unroll
    for (int i = 0; i < kStatRun; ++i) {
      const int p = p0 + i;
      const int v = (int)(__umul24(N, ss[i]) - __umul24(s[i], s[i]));
      // 1/sqrt(v) by the hardware reciprocal square root (within 1 ulp); zero
      // for a flat window, whose cost is then 1 at every disparity
      const float inv = v > 0 ? __builtin_amdgcn_rsqf((float)v) : 0.0f;
      if (ref) {
        if (p < W) {
          LR[p * RS + NP] = 0u - s[i];
          LR[p * RS + NP + 1] = __float_as_uint(inv);
          if (mode == kSums && blockIdx.x == 0) {
            if (a.s_l) a.s_l[(size_t)y * W + p] = (int)s[i];
            if (a.s_ll) a.s_ll[(size_t)y * W + p] = (int)ss[i];
          }
        }
      } else if (p < lay.nTS) {
        TR[p * RS + NP] = s[i];
        TR[p * RS + NP + 1] = __float_as_uint(inv);
        if (mode == kSums) {
          // each x' in [-(D-1), W-1] is written by exactly one chunk
          const int xe = p - P - d0;
          const bool own = (blockIdx.x == 0) ? (xe >= -P) : (xe <= -d0);
          if (own && xe >= -(a.D - 1) && xe <= W - 1) {
            const size_t idx = (size_t)y * (W + a.D - 1) + xe + a.D - 1;
            if (a.s_t) a.s_t[idx] = (int)s[i];
            if (a.s_tt) a.s_tt[idx] = (int)ss[i];
          }
        }
      }
    }
  }
}

// W_L(x) of row y for x in [0, W]; zero at both ends.
__device__ void stage_row_weights(const HArgs& a, float* WH, int y) {
  const uint8_t* g = a.guide + (size_t)y * a.pitch;
  for (int x = threadIdx.x; x <= a.W; x += blockDim.x)
    WH[x] = (x >= 1 && x < a.W) ? dt_weight(g[x], g[x - 1], a.inv_sigma_s, a.range_coef) : 0.0f;
}

// Cross-sum column of one window column for this lane's disparity, from the
// column's reference and target records: sum_k dot4(L pack, T pack).
template <int R>
__device__ __forceinline__ uint32_t colsum(const uint32_t* lrec, const uint32_t* trec) {
  constexpr int NP = packs_of(R);
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < NP; ++k) s = __builtin_amdgcn_udot4(lrec[k], trec[k], s, false);
  return s;
}

// cost = 1 - clamp(ZNCC, -1, 1) from the exact integer numerator
// l^2 S_RT - S_R S_T, given the records of the reference position and of the
// target position (words NP, NP+1: -S_R and 1/sigma_R, S_T and 1/sigma_T).
// For l <= 15, S_RT and the window sums are below 2^24 (exact operands of the
// 24-bit multiplies), the products l^2 S_RT and S_R S_T below 2^32, and the
// numerator below 2^31 in magnitude, so the wrapping 32-bit sum is exact.
template <int R>
__device__ __forceinline__ float zncc_cost_rec(uint32_t srt, const uint32_t* lrec, const uint32_t* trec) {
  constexpr int NP = packs_of(R);
  constexpr uint32_t N = (2 * R + 1) * (2 * R + 1);
  const int nsl = (int)lrec[NP], st = (int)trec[NP];
  const float il = __uint_as_float(lrec[NP + 1]), it = __uint_as_float(trec[NP + 1]);
  const int num = (int)(__umul24(N, srt) + (uint32_t)__mul24(nsl, st));
  const float c = fmaf(-(float)num, il * it, 1.0f);
  return fminf(fmaxf(c, 0.0f), 2.0f);
}

// ---------------------------------------------------------------------------
// Narrow working volumes.  The DT's gain ranges from ~1 per pass at edges to
// 1/(1-K) per pass in flat areas, so aggregated values spread over far more
// binades than FP16 holds.  An FP16 working volume is therefore stored scaled
// per pixel by a power of two taken from the pixel's gain G: the DT of an
// all-ones slice at the same stage (G >= 1; it depends only on the guide).
// The passes are linear with positive weights and every cost lies in [0, 2],
// so every value satisfies C <= 2 G; with k = floor(log2 G) the stored
// C * 2^(kGainBias - k) stays below 2^15 for every disparity, without any
// reduction over disparities.  Rescaling by a power of two is exact, so only
// the FP16 rounding remains (relative 2^-11 down to C / G ~ 2^-28).  Each
// workgroup computes the G line it needs with one wave (line_pair_gain); the
// workgroup of disparity chunk 0 also writes it for the next stage.  BF16 and
// FP32 volumes store plain values.
// ---------------------------------------------------------------------------

// Maximum of a non-negative 32-bit key over the 64 lanes (result from lane 63).
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast:15
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Minimum of a 32-bit key over the 64 lanes (result from lane 63).
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  const int id = -1;  // identity for lanes without a source
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0xB1, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x4E, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x141, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x140, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x142, 0xA, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x143, 0xC, 0xF, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Wave minimum of B independent keys at once (results in lane 63): the six DPP
// steps of wave_min_u32 applied stage by stage across the block, so no step
// waits on the one just before it.
template <int B>
__device__ __forceinline__ void block_min_u32(uint32_t (&m)[B]) {
  const int id = -1;
#define ZDT_STAGE(CTRL, ROWMASK)                                                                     \
  _Pragma("unroll") for (int i = 0; i < B; ++i) m[i] =                                              \
      min(m[i], (uint32_t)__builtin_amdgcn_update_dpp(id, (int)m[i], CTRL, ROWMASK, 0xF, false));
  ZDT_STAGE(0xB1, 0xF)   // quad_perm [1,0,3,2]
  ZDT_STAGE(0x4E, 0xF)   // quad_perm [2,3,0,1]
  ZDT_STAGE(0x141, 0xF)  // row_half_mirror
  ZDT_STAGE(0x140, 0xF)  // row_mirror
  ZDT_STAGE(0x142, 0xA)  // row_bcast:15
  ZDT_STAGE(0x143, 0xC)  // row_bcast:31
#undef ZDT_STAGE
}

// Scale factors of a gain G >= 1 with e = floor(log2 G): 2^(e - kGainBias) to
// decode a stored value and 2^(kGainBias - e) to encode one.  Multiplying by
// them equals ldexp by the same exponents, bit for bit.
__device__ __forceinline__ float gain_scale_in(float g) {
  return __uint_as_float(((__float_as_uint(g) >> 23) - kGainBias) << 23);
}
__device__ __forceinline__ float gain_scale_out(float g) {
  return __uint_as_float((uint32_t)(254 + kGainBias - (int)(__float_as_uint(g) >> 23)) << 23);
}

// Exclusive scan over the 64 lanes, in lane order, of the affine maps
// c -> A c + B: the composition of the maps of lanes 0..l-1 (identity for lane
// 0), as DPP row shifts and row broadcasts (identity where a lane has no
// source).
__device__ __forceinline__ float lane_carry(float A, float B) {
  const int one = __float_as_int(1.0f);
#define ZDT_STEP(CTRL, ROWMASK)                                                                    \
  {                                                                                                \
    const float pa = __int_as_float(__builtin_amdgcn_update_dpp(one, __float_as_int(A), CTRL, ROWMASK, 0xF, false)); \
    const float pb = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(B), CTRL, ROWMASK, 0xF, false));   \
    B = fmaf(A, pb, B);                                                                            \
    A *= pa;                                                                                       \
  }
  ZDT_STEP(0x111, 0xF)  // row_shr:1
  ZDT_STEP(0x112, 0xF)  // row_shr:2
  ZDT_STEP(0x114, 0xF)  // row_shr:4
  ZDT_STEP(0x118, 0xF)  // row_shr:8
  ZDT_STEP(0x142, 0xA)  // row_bcast:15
  ZDT_STEP(0x143, 0xC)  // row_bcast:31
#undef ZDT_STEP
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(B), 0x138, 0xF, 0xF, false));  // wave_shr:1
}

// The L-then-R pass pair (or U-then-D) of one line of n values, run by one
// whole wave: out = pair(in) with in = 1 everywhere when `in` is NULL; w[i] is
// the forward weight into i (w[0] = w[n] = 0), the backward weight into i is
// w[i + 1].  The line is cut into 64 blocks of ceil(n / 64) values; lane l
// takes block l for the forward pass and block 63 - l for the backward one, so
// both passes compose their block carries with the same forward lane scan.
// `in` and `out` are LDS lines.
__device__ void line_pair_gain(const float* in, float* out, const float* w, int n) {
  const int lane = threadIdx.x & (kWave - 1);
  const int m = (n + kWave - 1) / kWave;
  int j0 = min(lane * m, n), j1 = min(j0 + m, n);
  float ell = 0.0f, P = 1.0f;
#pragma unroll 4
  for (int j = j0; j < j1; ++j) {
    ell = fmaf(w[j], ell, in ? in[j] : 1.0f);
    P *= w[j];
  }
  float prev = lane_carry(P, ell);
#pragma unroll 4
  for (int j = j0; j < j1; ++j) {
    prev = fmaf(w[j], prev, in ? in[j] : 1.0f);
    out[j] = prev;
  }
  j0 = min((kWave - 1 - lane) * m, n);
  j1 = min(j0 + m, n);
  ell = 0.0f;
  P = 1.0f;
#pragma unroll 4
  for (int j = j1 - 1; j >= j0; --j) {
    ell = fmaf(w[j + 1], ell, out[j]);
    P *= w[j + 1];
  }
  prev = lane_carry(P, ell);
#pragma unroll 4
  for (int j = j1 - 1; j >= j0; --j) {
    prev = fmaf(w[j + 1], prev, out[j]);
    out[j] = prev;
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin by linear id, and each
// XCD has its own L2.  The tiles of a pass (line, disparity chunk), line-major,
// are dealt so that every XCD takes one contiguous range of them: the chunks of
// one line (which share the line's guide pixels, gains and, in 16-bit volumes
// with 32-lane segments, the two halves of each 128-byte volume line) and
// neighbouring lines (which share the 128-byte lines of the column-strided
// guide and gain maps in the V pass) then meet in one L2.  The grid is
// kXcds * ceil(ntiles / kXcds) workgroups; `valid` is false for the padding.
constexpr int kXcds = 8;
struct Tile {
  int line, chunk;
  bool valid;
};
__host__ __device__ inline int xcd_grid(int ntiles) { return kXcds * ((ntiles + kXcds - 1) / kXcds); }
__device__ __forceinline__ Tile xcd_tile(int L, int ntiles, int nchunks) {
  const int per = (ntiles + kXcds - 1) / kXcds;
  const int t = (L % kXcds) * per + L / kXcds;
  return {t / nchunks, t % nchunks, t < ntiles};
}
// The 16-bit H passes instead only put the two chunks that hold the halves of
// the same 128-byte lines (2p and 2p+1) on one XCD, at linear ids L and L + 8,
// and keep the lines in order across XCDs (measured a little faster there).
__host__ __device__ inline int pair_grid(int nlines, int nchunks) { return (nlines * ((nchunks + 1) / 2) + 7) / 8 * 16; }
__device__ __forceinline__ Tile pair_tile(int L, int nlines, int nchunks) {
  const int npairs = (nchunks + 1) / 2;
  const int r = L & 15;
  const int i = (L >> 4) * 8 + (r & 7);
  const Tile t{i / npairs, 2 * (i % npairs) + (r >> 3), true};
  return {t.line, t.chunk, t.line < nlines && t.chunk < nchunks};
}
// Which tile order an H pass uses (measured per element size at 1280x384,
// D = 128 and 1920x1080, D = 256): pair_tile for 16-bit volumes, xcd_tile for
// the others.  Every V pass uses xcd_tile (a column's chunks and neighbouring
// columns in one L2; at 1920x1080 the FP32 U/D pair runs 8 % faster than in
// the plain order of a (chunk, column) grid).
template <int BYTES>
constexpr int h_order() { return BYTES == 2 ? 1 : 2; }  // 1: pair_tile, 2: xcd_tile

// Waves per SIMD the register allocator is asked to allow.  H pairs with two
// segments of up to 40 values per wave are held to 64 VGPRs (spilling a few
// words at most), so two 1024-lane workgroups share a CU and one's staging and
// exchanges overlap the other's recursions; the rest get up to 128 VGPRs.
template <int R, int SEG, int LPS, int MODE>
constexpr int h_waves_per_eu() {
  return ((MODE == kCostHPair || MODE == kHPair) && LPS == 32 && SEG <= 40) ? 8 : 4;
}

template <int R, int SEG, int LPS, typename T, int MODE>
__global__ __launch_bounds__(1024, (h_waves_per_eu<R, SEG, LPS, MODE>())) void hpass_kernel(HArgs args, HJobs jobs) {
  extern __shared__ uint32_t smem[];
  HArgs a = args;
  {
    const HJob& jb = jobs.j[blockIdx.z];
    a.left = jb.left;
    a.right = jb.right;
    a.guide = jb.guide;
    a.vol = jb.vol;
    a.g_in = jb.g_in;
    a.g_out = jb.g_out;
    a.ref = jb.ref;
  }
  constexpr int NW = 2 * R + 1;  // window side
  constexpr int SPW = kWave / LPS;  // segments per wave
  constexpr bool kZncc = MODE != kHPair;
  constexpr bool kDT = MODE == kCostHPair || MODE == kHPair;
  constexpr bool kHalf = std::is_same<T, f16x>::value;  // gain-scaled FP16
  constexpr bool kInt = is_int_vol<T>();                 // T-scaled integer volume (Sec. IV-C)
  static_assert(LPS == 64 || LPS == 32, "lanes per segment");
  constexpr uint32_t kBytes = sizeof(T);
  int y, chunk;
  if constexpr (kDT) {
    const Tile t = h_order<kBytes>() == 1 ? pair_tile(blockIdx.x, a.H, a.nchunks)
                                          : xcd_tile(blockIdx.x, a.H * a.nchunks, a.nchunks);
    if (!t.valid) return;  // padding of the grid
    y = __builtin_amdgcn_readfirstlane(t.line);  // the workgroup's tile, in SGPRs
    chunk = __builtin_amdgcn_readfirstlane(t.chunk);
  } else {
    y = blockIdx.y;
    chunk = blockIdx.x;
  }
  const int d0 = chunk * LPS;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int dloc = lane & (LPS - 1);
  const int seg = wave * SPW + (SPW == 1 ? 0 : lane / LPS);
  const int d = d0 + dloc;
  const bool active = d < a.D;
  const int W = a.W, D = a.D;
  // Two segments per wave are only used when the row splits into full segments
  // of exactly SEG values (checked by the host), so every step is in the row.
  constexpr bool kFull = LPS == 32;
  // Register-resident modes size LDS for the widest row of the instance, so the
  // array offsets are compile-time constants (one base register per index
  // pattern instead of one per array); streaming modes size it for this row.
  constexpr int kWMax = (kWave / LPS) * kMaxWaves * SEG;
  const HLayout lay = h_layout(kDT ? kWMax : W, R, LPS, SEG, kZncc, kDT, kHalf || kInt);
  if constexpr (kZncc) stage_zncc<R, LPS>(a, lay, smem, y, d0, MODE);
  if constexpr (kDT) stage_row_weights(a, (float*)(smem + lay.oWH), y);
  float* GI = (float*)(smem + lay.oGI);
  float* GO = (float*)(smem + lay.oGO);
  float* SI = (float*)(smem + lay.oSI);
  if constexpr (kHalf && MODE == kHPair) {
    const float* gr = a.g_in + (size_t)y * W;  // gains of the stored input row
    for (int x = threadIdx.x; x < W; x += blockDim.x) {
      const float g = gr[x];
      GI[x] = g;
      SI[x] = gain_scale_in(g);
    }
  }
  if constexpr (kInt && MODE == kCostHPair) {
    if (a.ref_role == kRefL2RIn) {
      const float* rr = a.ref + (size_t)y * W;  // the row's stored L2R output at d = 0
      for (int x = threadIdx.x; x < W; x += blockDim.x) GI[x] = rr[x];
    }
  }
  __syncthreads();

  // segment [x0, x0 + len)
  const int x0 = seg * a.segl;
  const int len = kFull ? SEG : min(a.segl, W - x0);
  const uint32_t rowbytes = (uint32_t)W * D * kBytes;
  const uint32_t xstride = (uint32_t)D * kBytes;
  const rsrc_t vrs = make_rsrc((const char*)a.vol + (size_t)y * rowbytes, rowbytes);
  const uint32_t voff = ((uint32_t)x0 * D + (uint32_t)(active ? d : D - 1)) * kBytes;
  // uniform offset of step k, clamped into the segment
  auto step_soff = [&](int k) -> uint32_t { return (uint32_t)(kFull ? k : min(k, len - 1)) * xstride; };

  // column records of position x0 (reference) and of its target at this
  // lane's disparity; position x0+k and window column x0+k-R+i sit k and k+i
  // records further on
  constexpr int RS = rec_words(R);
  uint32_t lo = lay.oLP + x0 * RS, to = lay.oTP + (x0 + LPS - 1 - dloc) * RS;
  // opaque offsets: one base register each, every record read at a small
  // constant offset from it (instead of rebasing each read pair)
  asm volatile("" : "+v"(lo), "+v"(to));
  const uint32_t* lrec = smem + lo;
  const uint32_t* trec = smem + to;

  if constexpr (MODE == kSums || MODE == kCost) {
    static_assert(LPS == 64, "streaming modes use one segment per wave");
    if (MODE == kSums && a.s_rt == nullptr) return;
    T* vol = (T*)a.vol;
    const size_t rowbase = (size_t)y * W * D;
    // running window: ring[s] holds the column sums of columns x0-R+s (mod NW)
    uint32_t ring[NW];
    uint32_t S = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      ring[i] = colsum<R>(lrec + i * RS, trec + i * RS);
      S += ring[i];
    }
    for (int kb = 0; kb < len; kb += NW) {
#pragma unroll
      for (int u = 0; u < NW; ++u) {
        const int k = kb + u;
        if (k < len) {
          const int x = x0 + k;
          if (k > 0) {
            const int slot = (u + NW - 1) % NW;
            const uint32_t cn = colsum<R>(lrec + (k + 2 * R) * RS, trec + (k + 2 * R) * RS);
            S = S + cn - ring[slot];
            ring[slot] = cn;
          }
          if (active) {
            const size_t idx = rowbase + (size_t)x * D + d;
            if constexpr (MODE == kSums) {
              a.s_rt[idx] = (int32_t)S;
            } else {
              const float c = zncc_cost_rec<R>(S, lrec + k * RS, trec + k * RS);
              Elem<T>::store(vol + idx, c * a.out_scale);
            }
          }
        }
      }
    }
    return;
  } else {
    const float* WH = (const float*)(smem + lay.oWH);
    float* EX = (float*)(smem + lay.oEX);
    float* EXS = (float*)(smem + lay.oEXS);
    float* EX2 = (float*)(smem + lay.oEX2);
    float* EXS2 = (float*)(smem + lay.oEXS2);
    constexpr bool scaled = kHalf;
    if constexpr (scaled) {
      // the row's gain after this pair, by the last wave; the other waves
      // start their segments meanwhile and read it only after two barriers
      if (wave == (int)(blockDim.x / kWave) - 1) {
        line_pair_gain(MODE == kHPair ? GI : nullptr, GO, WH, W);
        for (int x = lane; x < W; x += kWave) {
          const float g = GO[x];
          if (chunk == 0) a.g_out[(size_t)y * W + x] = g;
          GO[x] = gain_scale_out(g);
        }
      }
    }
    // W_L at x0 + k (padded past the row), from an opaque base so that every
    // step reads at a small constant offset
    uint32_t wo = lay.oWH + x0;
    asm volatile("" : "+v"(wo));
    const float* wp = (const float*)(smem + wo);
    float c[SEG];
    // ---- loop A: values of the segment + carry-free L pass (ell) and weight product P
    float ell = 0.0f, P = 1.0f;
    if constexpr (MODE == kCostHPair) {
      // Two sweeps over the segment keep the peak register count down: first
      // the window cross-sums S_RT (running over a ring of column sums), held
      // as bits in c[], then the costs and the carry-free L pass.
      uint32_t ring[NW];
      uint32_t S = 0;
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        ring[i] = colsum<R>(lrec + i * RS, trec + i * RS);
        S += ring[i];
      }
#pragma unroll
      for (int k = 0; k < SEG; ++k) {
        if (k > 0) {
          const int slot = (k - 1) % NW;
          const uint32_t cn = colsum<R>(lrec + (k + 2 * R) * RS, trec + (k + 2 * R) * RS);
          S = S + cn - ring[slot];
          ring[slot] = cn;
        }
        c[k] = __uint_as_float(S);
        if (k % 2 == 1) {
          pin(S);
          fence();
        }
      }
      fence();
#pragma unroll
      for (int k = 0; k < SEG; ++k) {
        const bool in = k < len;
        c[k] = zncc_cost_rec<R>(__float_as_uint(c[k]), lrec + k * RS, trec + k * RS);
        if constexpr (kInt) c[k] *= a.cost_scale;
        const float w = wp[k];
        ell = in ? fmaf(w, ell, c[k]) : ell;
        P = in ? P * w : P;
        if (k % 4 == 3) {
          pin(ell, P);
          fence();
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < SEG; ++k) c[k] = Elem<T>::bload(vrs, voff, step_soff(k));
      __builtin_amdgcn_sched_barrier(0);
      const float* si = SI + x0;  // input scale factors at x0 + k
#pragma unroll
      for (int k = 0; k < SEG; ++k) {
        const bool in = k < len;
        if constexpr (scaled) c[k] *= si[k];
        const float w = wp[k];
        ell = in ? fmaf(w, ell, c[k]) : ell;
        P = in ? P * w : P;
        step_fence(k, ell, P);
      }
    }
    // every lane stores its segment's weight product (one value per segment):
    // a single-lane store lets the compiler defer the product chain and keep
    // the whole line of weights live until then
    EX[seg * LPS + dloc] = ell;
    EXS[seg] = P;
    __syncthreads();
    const float carry = carry_in<false>(EX, EXS, seg, a.nseg, LPS, dloc, min(wave * SPW + SPW - 1, a.nseg - 1));
    reload_fence();
    // ---- loop B: exact L pass from the true carry; accumulate the carry-free R value at x0
    // Integer volumes: the R pass reads the L2R output as stored (rounded to
    // an int16; the L recursion itself runs on unrounded values), normalized
    // in the first sweep of Int8 (R2L) by the stored d = 0 slice.
    float prev = carry, acc = 0.0f, pi = 1.0f;
    const float* rl = GI + x0;  // Int8 first sweep: the L2R output's d = 0 slice at x0 + k
    [[maybe_unused]] const bool sub_ref = kInt && MODE == kCostHPair && a.ref_role == kRefL2RIn;
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      const bool in = k < len;
      const float w = wp[k];
      const float cl = fmaf(w, prev, c[k]);
      float cv = cl;
      if constexpr (kInt) {
        cv = rq16(cl);
        if (sub_ref) cv -= rl[k];
      }
      c[k] = in ? cv : c[k];
      prev = in ? cl : prev;
      if (k > 0) pi = in ? pi * w : pi;
      acc = in ? fmaf(cv, pi, acc) : acc;
      step_fence(k, prev, acc, pi);
    }
    if constexpr (kInt && MODE == kCostHPair) {
      if (a.ref_role == kRefL2ROut) {  // Int8 reference launch: the stored L2R output at d = 0
#pragma unroll
        for (int k = 0; k < SEG; ++k)
          if (d == 0 && k < len) a.ref[(size_t)y * W + x0 + k] = c[k];
        return;
      }
    }
    const float Q = pi * WH[x0 + len];
    EX2[seg * LPS + dloc] = acc;
    EXS2[seg] = Q;
    __syncthreads();
    const float kappa = carry_in<true>(EX2, EXS2, seg, a.nseg, LPS, dloc, max(a.nseg - 1 - wave * SPW, 0));
    reload_fence();
    // ---- loop D: exact R pass from the true carry; each value is stored as
    // soon as it is final, which spreads a workgroup's stores over the loop
    float next = kappa;
    const float* so = GO + x0;  // output scale factors at x0 + k
    // Lanes past the last disparity, and steps past a ragged segment, store
    // at a lane offset beyond the row's buffer range, which the buffer unit
    // discards (its range check covers the lane offset, not the step offset),
    // so the stores need no branch.
    constexpr uint32_t kDrop = 0x80000000u;
    const uint32_t voff_st = active ? voff : kDrop;
#pragma unroll
    for (int k = SEG - 1; k >= 0; --k) {
      const bool in = k < len;
      const float cr = fmaf(wp[k + 1], next, c[k]);
      next = in ? cr : next;
      const float v = scaled ? cr * so[k] : cr * a.out_scale;
      Elem<T>::bstore(vrs, in ? voff_st : kDrop, step_soff(k), v);
      if constexpr (kInt && MODE == kCostHPair)
        if (a.ref_role == kRefR2LOut && d == 0 && in) a.ref[(size_t)y * W + x0 + k] = rq16(v);
      step_fence(SEG - 1 - k, next);
    }
  }
}

// ---------------------------------------------------------------------------
// V pair (+ optional WTA)
// ---------------------------------------------------------------------------
struct VArgs {
  const uint8_t* guide;
  int pitch, W, H, D;
  float inv_sigma_s, range_coef, out_scale;
  int ref_sub;         // Int16 first sweep: subtract `ref` (U2D normalization, Eq. DT_new)
  void* vol;
  const float* g_in;   // FP16 working volume: gain map [H][W] of the stored input
  float* g_out;        // and of the output (not for the WTA pass)
  int32_t* disp;       // WTA with a single chunk: final disparity
  float* part_val;     // WTA with several chunks: [chunk][W][H] minimum (column-major)
  int32_t* part_idx;   // and its disparity
  const float* ref;    // Int16: [H][W] stored R2L output at d = 0 (written by the first H pair)
  int segl, nseg;      // segment length and number of segments of a column
  int nchunks;         // disparity chunks of LPS lanes
};

struct VJob {
  const uint8_t* guide;
  void* vol;
  const float* g_in;
  float* g_out;
  int32_t* disp;
  float* part_val;
  int32_t* part_idx;
  const float* ref;
};
struct VJobs {
  VJob j[kMaxJobs];
};

// WV[H+1] (+ SEG spare entries), EX/EX2 [32 segments x 32 lanes or 16 x 64],
// EXS/EXS2 [kMaxSegs], and for the FP16 working volume GI, GO, SI [H + SEG],
// the column's gains before and after the pair and the input scale factors;
// integer volumes use GI for the column of the normalization map.
__host__ __device__ inline int v_lds_words(int H, int SEG, bool scaled, bool ints) {
  return (H + 1 + SEG) + 2 * (kMaxWaves * kWave + kMaxSegs) + (scaled ? 3 * (H + SEG) : (ints ? H + SEG : 0));
}

// Order-preserving 32-bit key of a float (-0 folded onto +0) and its inverse.
__device__ __forceinline__ uint32_t order_key(float v) {
  const uint32_t u = __float_as_uint(v + 0.0f);
  return (u >> 31) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_value(uint32_t k) { return __uint_as_float((k >> 31) ? (k & 0x7FFFFFFFu) : ~k); }

// Wave (LANES = 64) or half-wave (LANES = 32) minimum of B independent keys at
// once; the result is in lane 63 (and lane 31 for the lower half-wave).
template <int B, int LANES>
__device__ __forceinline__ void group_min_u32(uint32_t (&m)[B]) {
  if constexpr (LANES == 64) {
    block_min_u32<B>(m);
  } else {
    const int id = -1;
#define ZDT_STAGE(CTRL, ROWMASK)                                                                     \
  _Pragma("unroll") for (int i = 0; i < B; ++i) m[i] =                                              \
      min(m[i], (uint32_t)__builtin_amdgcn_update_dpp(id, (int)m[i], CTRL, ROWMASK, 0xF, false));
    ZDT_STAGE(0xB1, 0xF)   // quad_perm [1,0,3,2]
    ZDT_STAGE(0x4E, 0xF)   // quad_perm [2,3,0,1]
    ZDT_STAGE(0x141, 0xF)  // row_half_mirror
    ZDT_STAGE(0x140, 0xF)  // row_mirror
    ZDT_STAGE(0x142, 0xA)  // row_bcast:15
#undef ZDT_STAGE
  }
}

// ---------------------------------------------------------------------------
// Butterfly minimum for the WTA of 64-lane segments.  A wave holds N pixels in
// N registers (lane = disparity); reducing each over 64 lanes separately costs
// six DPP steps per pixel.  Here the registers are merged pairwise instead,
// six times: each merge takes the minimum over half of the remaining lanes of
// two registers' pixels at once and keeps one pixel in each half of the lanes
// (permlane32 / permlane16 swaps for the first two stages, then DPP row_ror:8,
// row_half_mirror, quad_perm xor 2 and xor 1 with a lane select).  After six
// stages every lane of the ceil-halved registers holds one pixel's minimum over
// all 64 lanes; bfly_map() gives, at compile time, the register and lane of
// each pixel.  An odd register is merged with itself.
// ---------------------------------------------------------------------------
constexpr int bfly_count(int n, int stages) { return stages == 0 ? n : bfly_count((n + 1) / 2, stages - 1); }

template <int N>
struct BflyMap {
  int reg[N], lane[N];
};

// Label (pixel index) of every lane of every register through the six stages.
template <int N>
constexpr BflyMap<N> bfly_map() {
  int lab[N][64] = {};
  int nl[N][64] = {};
  for (int r = 0; r < N; ++r)
    for (int l = 0; l < 64; ++l) lab[r][l] = r;
  int n = N;
  for (int st = 1; st <= 6; ++st) {
    const int m = (n + 1) / 2;
    for (int i = 0; i < m; ++i) {
      const int A = 2 * i, B = 2 * i + 1 < n ? 2 * i + 1 : 2 * i;
      for (int l = 0; l < 64; ++l) {
        int v = 0;
        if (st == 1) v = l < 32 ? lab[A][l] : lab[B][l];
        else if (st == 2) v = (l / 16) % 2 == 0 ? lab[A][l] : lab[B][l - 16];
        else v = (l % (32 >> (st - 2))) < (16 >> (st - 2)) ? lab[A][l] : lab[B][l];
        nl[i][l] = v;
      }
    }
    for (int i = 0; i < m; ++i)
      for (int l = 0; l < 64; ++l) lab[i][l] = nl[i][l];
    n = m;
  }
  BflyMap<N> out{};
  for (int k = 0; k < N; ++k) {
    out.reg[k] = -1;
    for (int r = n - 1; r >= 0; --r)
      for (int l = 63; l >= 0; --l)
        if (lab[r][l] == k) {
          out.reg[k] = r;
          out.lane[k] = l;
        }
  }
  return out;
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_min_u32(uint32_t v) {
  return min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, CTRL, 0xF, 0xF, false));
}

// One merge stage over n registers in place (results in r[0 .. ceil(n/2) - 1]).
template <int ST, int N>
__device__ __forceinline__ void bfly_stage(uint32_t (&r)[N], int n, int lane) {
#pragma unroll
  for (int i = 0; i < (N + 1) / 2; ++i) {
    if (i >= (n + 1) / 2) break;
    const uint32_t a = r[2 * i];
    const bool pair = 2 * i + 1 < n;
    const uint32_t b = pair ? r[2 * i + 1] : a;
    uint32_t y;
    if constexpr (ST == 1 || ST == 2) {
      const auto p = ST == 1 ? __builtin_amdgcn_permlane32_swap(a, b, false, false)
                             : __builtin_amdgcn_permlane16_swap(a, b, false, false);
      y = min((uint32_t)p[0], (uint32_t)p[1]);
    } else {
      constexpr int CTRL = ST == 3 ? 0x128 : ST == 4 ? 0x141 : ST == 5 ? 0x4E : 0xB1;
      constexpr int SPAN = 32 >> (ST - 2), HALF = SPAN / 2;  // 16/8, 8/4, 4/2, 2/1
      // both DPP minima are taken with every lane active, before the select:
      // left to itself the compiler may turn the select into a branch and run
      // the second one with half the lanes off, whose values it then cannot read
      uint32_t ma = dpp_min_u32<CTRL>(a), mb = pair ? dpp_min_u32<CTRL>(b) : ma;
      pin(ma, mb);
      y = (lane % SPAN) < HALF ? ma : mb;
    }
    r[i] = y;
  }
}

// V pair (U then D, Eqs. DT3-DT4) of one column x and one chunk of LPS
// disparities, optionally followed by the WTA.  A wave holds 64 / LPS segments
// of the column, each LPS lanes wide (consecutive disparities).  FULL: every
// segment holds exactly SEG rows (checked by the host; required for LPS = 32).
// Tiles (column, chunk) are dealt in the XCD-contiguous order of xcd_tile, so
// the workgroups of a column's chunks and of neighbouring columns share an L2.
//
// Waves per SIMD the register allocator is asked to allow.  Two 32-lane
// segments of up to 36 rows per wave are held to 64 VGPRs, so two 15-wave
// workgroups of a 1080-row column share a CU (without the bound the 16-bit
// loads and their FP32 values are both kept live and one workgroup fills the
// CU); so are the gain-scaled FP16 U/D pairs with 64-lane segments of up to 48
// rows (four 8-wave workgroups per CU instead of three).  The integer
// volumes' 64-lane pairs of up to 48 rows take 8 waves, 6 with the WTA (three
// workgroups per CU instead of two; 80 VGPRs and a 16-byte spill, measured
// 6-10 % faster); their 32-lane pairs keep the default (under the bound their
// codecs spill).
template <int SEG, int LPS, bool WTA, typename T>
constexpr int v_waves_per_eu() {
  if constexpr (is_int_vol<T>()) return (LPS == 64 && SEG <= 48) ? (WTA ? 6 : 8) : 4;
  if constexpr (LPS == 32 && SEG <= 36) return 8;
  return (LPS == 64 && SEG <= 48 && !WTA && std::is_same<T, f16x>::value) ? 8 : 4;
}

template <int SEG, bool FULL, typename T, int LPS, bool WTA>
__global__ __launch_bounds__(1024, (v_waves_per_eu<SEG, LPS, WTA, T>())) void vpass_kernel(VArgs args, VJobs jobs) {
  extern __shared__ uint32_t smem[];
  VArgs a = args;
  {
    const VJob& jb = jobs.j[blockIdx.z];
    a.guide = jb.guide;
    a.vol = jb.vol;
    a.g_in = jb.g_in;
    a.g_out = jb.g_out;
    a.disp = jb.disp;
    a.part_val = jb.part_val;
    a.part_idx = jb.part_idx;
    a.ref = jb.ref;
  }
  constexpr bool kHalf = std::is_same<T, f16x>::value;  // gain-scaled FP16
  constexpr bool kInt = is_int_vol<T>();                 // T-scaled integer volume
  static_assert(LPS == 64 || (LPS == 32 && FULL), "two segments per wave need full segments");
  constexpr int SPW = kWave / LPS;
  constexpr uint32_t kBytes = sizeof(T);
  const Tile t = xcd_tile(blockIdx.x, a.W * a.nchunks, a.nchunks);
  if (!t.valid) return;  // padding of the grid
  // the tile is the workgroup's: kept in SGPRs (the division leaves it in VGPRs)
  const int x = __builtin_amdgcn_readfirstlane(t.line), chunk = __builtin_amdgcn_readfirstlane(t.chunk);
  const int d0 = chunk * LPS;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int dloc = lane & (LPS - 1);
  const int seg = wave * SPW + (SPW == 1 ? 0 : lane / LPS);
  const int d = d0 + dloc;
  const bool act = d < a.D;
  const int W = a.W, H = a.H, D = a.D;
  float* WV = (float*)smem;
  float* EX = WV + (H + 1 + SEG);
  float* EXS = EX + kMaxWaves * kWave;
  float* EX2 = EXS + kMaxSegs;
  float* EXS2 = EX2 + kMaxWaves * kWave;
  float* GI = EXS2 + kMaxSegs;
  float* GO = GI + (H + SEG);  // gains, then output scale factors (see the H pass)
  float* SI = GO + (H + SEG);  // input scale factors
  if constexpr (kHalf)
    for (int y = threadIdx.x; y < H; y += blockDim.x) {
      const float g = a.g_in[(size_t)y * W + x];
      GI[y] = g;
      SI[y] = gain_scale_in(g);
    }
  if constexpr (kInt)
    if (a.ref_sub)
      for (int y = threadIdx.x; y < H; y += blockDim.x) GI[y] = a.ref[(size_t)y * W + x];
  for (int y = threadIdx.x; y <= H; y += blockDim.x)
    WV[y] = (y >= 1 && y < H) ? dt_weight(a.guide[(size_t)y * a.pitch + x], a.guide[(size_t)(y - 1) * a.pitch + x],
                                          a.inv_sigma_s, a.range_coef)
                              : 0.0f;
  __syncthreads();
  const int y0 = seg * a.segl;
  const int len = FULL ? SEG : min(a.segl, H - y0);  // >= 1; wave-uniform
  const uint32_t rowbytes = (uint32_t)W * D * kBytes;
  // buffer over the volume from column x on; every offset below stays inside it
  // 32-bit offsets: the host admits volumes below 4 GiB
  const uint32_t col0 = (uint32_t)x * (uint32_t)D * kBytes;
  const rsrc_t vrs = make_rsrc((const char*)a.vol + col0, (uint32_t)H * W * D * kBytes - col0);
  constexpr bool scaled = kHalf;
  if constexpr (scaled && !WTA) {
    // the column's gain after this pair, by the last wave (read after two barriers)
    if (wave == (int)(blockDim.x / kWave) - 1) {
      line_pair_gain(GI, GO, WV, H);
      for (int y = lane; y < H; y += kWave) {
        const float g = GO[y];
        if (chunk == 0) a.g_out[(size_t)y * W + x] = g;
        GO[y] = gain_scale_out(g);
      }
    }
  }
  const float* si = SI + y0;  // input scale factors at y0 + k
  const float* wp = WV + y0;  // W_U at y0 + k; padded past the column
  // per-lane offset: the disparity, plus the segment's first row when the two
  // halves of a wave hold different segments; per-step offset: the row step
  const uint32_t voff = (uint32_t)(act ? d : D - 1) * kBytes + (SPW == 1 ? 0u : (uint32_t)y0 * rowbytes);
  auto step_off = [&](int k) -> uint32_t {
    if constexpr (SPW == 1) return (uint32_t)(y0 + (FULL || k < len ? k : len - 1)) * rowbytes;
    return (uint32_t)k * rowbytes;
  };

  // Values are loaded as raw bits and decoded in loop A, so each loaded
  // value's register is free once its FP32 value exists (loaded and decoded
  // at once, both sets were live together and the 64-VGPR bound of 36-row
  // segments spilled).
  float c[SEG];
#pragma unroll
  for (int k = 0; k < SEG; ++k) c[k] = __uint_as_float(Elem<T>::braw(vrs, voff, step_off(k)));
  __builtin_amdgcn_sched_barrier(0);
  // ---- loop A: carry-free U pass (decoding scaled FP16 values on the way;
  // Int16's first sweep subtracts the stored R2L output's d = 0 slice first)
  float ell = 0.0f, P = 1.0f;
  const float* rf = GI + y0;
  [[maybe_unused]] const bool sub_ref = kInt && a.ref_sub;
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    const bool in = k < len;
    const float w = wp[k];
    c[k] = Elem<T>::decode(__float_as_uint(c[k]));
    if constexpr (scaled) c[k] *= si[k];
    if constexpr (kInt)
      if (sub_ref) c[k] -= rf[k];
    ell = in ? fmaf(w, ell, c[k]) : ell;
    P = in ? P * w : P;
    step_fence(k, ell, P);
  }
  EX[seg * LPS + dloc] = ell;
  EXS[seg] = P;  // from every lane (see the H pass)
  __syncthreads();
  float prev;
  if constexpr (SPW == 1) {  // at most 15 segments before: a plain serial composition
    prev = 0.0f;
    for (int s = 0; s < seg; ++s) prev = fmaf(EXS[s], prev, EX[s * LPS + dloc]);
  } else {
    prev = carry_in<false>(EX, EXS, seg, a.nseg, LPS, dloc, min(wave * SPW + SPW - 1, a.nseg - 1));
  }
  reload_fence();
  // ---- loop B: exact U pass; carry-free D value at y0 (integer volumes: the
  // D pass reads the U2D output as stored, rounded to an int16)
  float acc = 0.0f, pi = 1.0f;
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    const bool in = k < len;
    const float w = wp[k];
    if (k > 0) pi = in ? pi * w : pi;
    const float cu = fmaf(w, prev, c[k]);
    const float cv = kInt ? rq16(cu) : cu;
    c[k] = in ? cv : c[k];
    prev = in ? cu : prev;
    acc = in ? fmaf(cv, pi, acc) : acc;
    step_fence(k, prev, acc, pi);
  }
  const float Q = pi * WV[y0 + len];
  EX2[seg * LPS + dloc] = acc;
  EXS2[seg] = Q;
  __syncthreads();
  float next;
  if constexpr (SPW == 1) {
    next = 0.0f;
    for (int s = a.nseg - 1; s > seg; --s) next = fmaf(EXS2[s], next, EX2[s * LPS + dloc]);
  } else {
    next = carry_in<true>(EX2, EXS2, seg, a.nseg, LPS, dloc, max(a.nseg - 1 - wave * SPW, 0));
  }
  reload_fence();
  // ---- loop D: exact D pass
#pragma unroll
  for (int k = SEG - 1; k >= 0; --k) {
    const bool in = k < len;
    const float cd = fmaf(wp[k + 1], next, c[k]);
    c[k] = in ? cd : c[k];
    next = in ? cd : next;
    step_fence(SEG - 1 - k, next);
  }
  if constexpr (!WTA) {
    const float* so = GO + y0;  // output scale factors at y0 + k
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      const float v = scaled ? c[k] * so[k] : c[k] * a.out_scale;
      if (k < len && act) Elem<T>::bstore(vrs, voff, step_off(k), v);
    }
  } else {
    // argmin over the chunk's disparities, lowest d on ties (Eq. WTA1).  The
    // aggregated costs are >= 0, so their bit patterns order like the values
    // (|.| folds a -0 onto +0); the centred integer volumes can be negative and
    // use the sign-aware key instead.  Idle lanes hold +inf.  64-lane
    // segments take all their pixels' minima in one butterfly; 32-lane ones
    // reduce 8 pixels at a time with their DPP chains interleaved.  Pixel k of
    // a segment keeps its (argmin, minimum) in lane k % LPS of that segment's
    // lanes, in result register k / LPS, and the results leave in one store
    // per register.
    auto key = [](float v) -> uint32_t {
      if constexpr (kInt) return order_key(v);
      return __float_as_uint(v) & 0x7FFFFFFFu;
    };
    const uint32_t kInf = key(__builtin_inff());
    constexpr int NR = (SEG + LPS - 1) / LPS;
    constexpr int B = 8;
    int rd[NR];
    uint32_t rv[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      rd[r] = 0;
      rv[r] = kInf;
    }
    if constexpr (LPS == 64) {
      // all SEG pixels' minima at once (butterfly), then per pixel the first
      // lane holding its minimum; pixel k's result goes to lane k % 64
      uint32_t u[SEG], t[SEG];
#pragma unroll
      for (int k = 0; k < SEG; ++k) {
        u[k] = act ? key(c[k]) : kInf;
        t[k] = u[k];
      }
      bfly_stage<1>(t, SEG, lane);
      bfly_stage<2>(t, bfly_count(SEG, 1), lane);
      bfly_stage<3>(t, bfly_count(SEG, 2), lane);
      bfly_stage<4>(t, bfly_count(SEG, 3), lane);
      bfly_stage<5>(t, bfly_count(SEG, 4), lane);
      bfly_stage<6>(t, bfly_count(SEG, 5), lane);
      constexpr BflyMap<SEG> map = bfly_map<SEG>();
#pragma unroll
      for (int k = 0; k < SEG; ++k) {
        if (k < len) {
          const uint32_t mk = (uint32_t)__builtin_amdgcn_readlane((int)t[map.reg[k]], map.lane[k]);
          const unsigned long long mask = __ballot(u[k] == mk);
          const int db = d0 + (int)__builtin_ctzll(mask);
          const bool mine = lane == k % 64;
          rd[k / 64] = mine ? db : rd[k / 64];
          rv[k / 64] = mine ? mk : rv[k / 64];
        }
      }
    }
    if constexpr (LPS != 64) {
      // two segments per wave: per pixel, a DPP minimum over each half-wave,
      // 8 pixels interleaved
#pragma unroll
      for (int k0 = 0; k0 < SEG; k0 += B) {
        uint32_t v[B], m[B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
          const int k = min(k0 + i, SEG - 1);
          v[i] = act ? key(c[k]) : kInf;
          m[i] = v[i];
        }
        group_min_u32<B, LPS>(m);
#pragma unroll
        for (int i = 0; i < B; ++i) {
          const int k = k0 + i;
          if (k < SEG && k < len) {
            const bool mine = dloc == k % LPS;
            const uint32_t mk0 = (uint32_t)__builtin_amdgcn_readlane((int)m[i], 31);
            const uint32_t mk1 = (uint32_t)__builtin_amdgcn_readlane((int)m[i], 63);
            const uint32_t mk = lane < 32 ? mk0 : mk1;
            const unsigned long long mask = __ballot(v[i] == mk);
            const int db0 = d0 + (int)__builtin_ctz((uint32_t)mask);
            const int db1 = d0 + (int)__builtin_ctz((uint32_t)(mask >> 32));
            rd[k / LPS] = mine ? (lane < 32 ? db0 : db1) : rd[k / LPS];
            rv[k / LPS] = mine ? mk : rv[k / LPS];
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int k = r * LPS + dloc;
      if (k < len) {
        const uint32_t p = (uint32_t)(y0 + k) * W + x;  // < W H
        if (a.disp) {
          a.disp[p] = rd[r];
        } else {
          // column-major partials: the wave's rows are consecutive words
          const uint32_t q = ((uint32_t)chunk * W + x) * H + (y0 + k);  // < ceil(D / 32) W H
          a.part_val[q] = kInt ? key_value(rv[r]) : __uint_as_float(rv[r]);
          a.part_idx[q] = rd[r];
        }
      }
    }
  }
}

// Combine per-chunk minima (chunks in increasing d; strict < keeps the lowest d).
struct WJob {
  const float* part_val;
  const int32_t* part_idx;
  int32_t* disp;
};
struct WJobs {
  WJob j[kMaxJobs];
};
// The partial minima are stored column-major ([chunk][x][y]: a V-pass wave's
// pixels are consecutive rows of one column); a 32 x 32 tile is combined with
// reads along y, transposed through LDS and written along x.  Block 32 x 8.
constexpr int kCombineTile = 32;
[[maybe_unused]] static __global__ void wta_combine_kernel(WJobs jobs, int nchunks, int W, int H) {
  __shared__ int32_t tile[kCombineTile][kCombineTile + 1];
  const WJob& jb = jobs.j[blockIdx.z];
  const int tx = threadIdx.x % kCombineTile, ty = threadIdx.x / kCombineTile;
  const int x0 = blockIdx.x * kCombineTile, y0 = blockIdx.y * kCombineTile;
  const size_t npix = (size_t)W * H;
#pragma unroll
  for (int j = ty; j < kCombineTile; j += 8) {
    const int x = x0 + j, y = y0 + tx;
    if (x < W && y < H) {
      // every chunk's minimum and disparity are loaded unconditionally, so all
      // the loads are in flight at once (no load waits on a comparison)
      const size_t q = (size_t)x * H + y;
      float best = jb.part_val[q];
      int idx = jb.part_idx[q];
#pragma unroll 4
      for (int c = 1; c < nchunks; ++c) {
        const float v = jb.part_val[c * npix + q];
        const int i = jb.part_idx[c * npix + q];
        idx = v < best ? i : idx;  // strict: the lower chunk (lower d) keeps a tie
        best = fminf(v, best);
      }
      tile[j][tx] = idx;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = ty; j < kCombineTile; j += 8) {
    const int y = y0 + j, x = x0 + tx;
    if (x < W && y < H) jb.disp[(size_t)y * W + x] = tile[tx][j];
  }
}

// Test entry of the 8-bit code: codes[i] = encode(in[i]), decoded[i] = decode(codes[i]).
[[maybe_unused]] static __global__ void i8_codec_kernel(const int16_t* in, uint8_t* codes, int16_t* decoded,
                                                        int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = i8_encode(in[i]);
  codes[i] = (uint8_t)c;
  decoded[i] = (int16_t)i8_decode(c);
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
  return v;
}

// Standalone WTA: each wave takes pixels p = global wave id, + total waves, ...
template <typename T>
__global__ __launch_bounds__(256) void wta_kernel(const T* vol, int npix, int D, int32_t* disp) {
  const int lane = threadIdx.x & (kWave - 1);
  const int gw = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nwaves = gridDim.x * blockDim.x / kWave;
  const float inf = __builtin_inff();
  for (int p = gw; p < npix; p += nwaves) {
    const T* c = vol + (size_t)p * D;
    float best = inf;
    int bd = 0;
    for (int dd = lane; dd < D; dd += kWave) {
      const float v = Elem<T>::load(c + dd);
      if (v < best) {
        best = v;
        bd = dd;
      }
    }
    const float m = wave_min(best);
    // among the lanes holding the minimum, the smallest of their own first d
    int cand = (best == m) ? bd : 0x7fffffff;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cand = min(cand, __shfl_xor(cand, off));
    if (lane == 0) disp[p] = cand;
  }
}

}  // namespace zdt
