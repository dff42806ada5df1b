/*
 * zdt_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU statement of what the stereo hot path
 * computes: ZNCC matching cost (Sec. III-A), domain-transform aggregation
 * (Sec. III-B, Eqs. DT1-DT4 with the weights of Eqs. k1-k4 and a), and
 * winner-take-all (Sec. III-C, Eq. WTA1).  Integers are int64, floating point
 * is IEEE double.  It shares no source, header or table with the HIP library;
 * only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it.
 *
 * Readings taken where the paper is silent or loose (each also listed in the
 * design notes of the repository):
 *   - left image = reference I_R, right image = target I_T, candidate I_T(x-d,y),
 *     d in [0, D) (Sec. III-A).
 *   - every pixel read is clamped to the image (replicate border), including
 *     target columns x-d+i < 0; the target window sums live on the extended
 *     column domain x' in [-(D-1), W-1].
 *   - a window of zero variance (exact integer test) gives ZNCC = 0, cost 1.
 *   - ZNCC is clamped to [-1, 1] (the text prints [0,1]; Cauchy-Schwarz gives
 *     [-1,1]); the aggregated quantity is the cost 1 - ZNCC and WTA takes its
 *     argmin, lowest d on ties (Eq. WTA1).
 *   - the DT weights come from the reference (left) image unless the caller
 *     asks for the target; intensity differences are in 0..255 units and
 *     sigma_r is given in intensity/255 units, so the exponent is
 *     -1/sigma_s - |dI| / (255 sigma_r)  (Eq. weight, a = exp(-1/sigma_s)).
 *   - W_R(x) = W_L(x+1) and W_D(y) = W_U(y+1) (Eqs. k1-k4); boundaries
 *     C_L(0)=C(0), C_R(W-1)=C_L(W-1), C_U(.,0)=C_R(.,0), C_D(.,H-1)=C_U(.,H-1).
 *   - "iterations": one L,R,U,D sweep is the paper's DT; I > 1 repeats the same
 *     four passes with the same weights on the previous sweep's output.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* I(u, v) with the replicate-border reading. */
static int pix(const uint8_t* img, int pitch, int W, int H, int u, int v) {
  return img[(ptrdiff_t)clampi(v, 0, H - 1) * pitch + clampi(u, 0, W - 1)];
}

/* ---------------------------------------------------------------------------
 * Window sums over the (2r+1)x(2r+1) window W centred on a pixel (Sec. IV-B,
 * Eq. sum1: S = sum of the pixel values of the window, computed directly).
 * S_L, S_LL : reference sums of I and I^2 at (x, y), arrays [H][W].
 * S_T, S_TT : target sums at (x', y) for x' in [-(D-1), W-1], arrays
 *             [H][W + D - 1] indexed by x' + D - 1.
 * ------------------------------------------------------------------------- */
int oracle_window_sums(const uint8_t* L, const uint8_t* R, int pitch, int W, int H, int D, int r,
                       int64_t* S_L, int64_t* S_LL, int64_t* S_T, int64_t* S_TT) {
  if (W < 1 || H < 1 || D < 1 || r < 0 || pitch < W) return -1;
  const int WE = W + D - 1;
  for (int y = 0; y < H; ++y) {
    for (int x = 0; x < W; ++x) {
      int64_t s = 0, ss = 0;
      for (int j = -r; j <= r; ++j)
        for (int i = -r; i <= r; ++i) {
          int64_t v = pix(L, pitch, W, H, x + i, y + j);
          s += v;
          ss += v * v;
        }
      S_L[(ptrdiff_t)y * W + x] = s;
      S_LL[(ptrdiff_t)y * W + x] = ss;
    }
    for (int xe = -(D - 1); xe < W; ++xe) {
      int64_t s = 0, ss = 0;
      for (int j = -r; j <= r; ++j)
        for (int i = -r; i <= r; ++i) {
          int64_t v = pix(R, pitch, W, H, xe + i, y + j);
          s += v;
          ss += v * v;
        }
      S_T[(ptrdiff_t)y * WE + xe + D - 1] = s;
      S_TT[(ptrdiff_t)y * WE + xe + D - 1] = ss;
    }
  }
  return 0;
}

/* Cross sum  S_RT(x,y,d) = sum over the window of I_R(x+i,y+j) * I_T(x-d+i,y+j)
 * (the Pi_RT term of Eq. OP_ZNCC), brute force, array [H][W][D]. */
int oracle_cross_sums(const uint8_t* L, const uint8_t* R, int pitch, int W, int H, int D, int r,
                      int64_t* S_RT) {
  if (W < 1 || H < 1 || D < 1 || r < 0 || pitch < W) return -1;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x)
      for (int d = 0; d < D; ++d) {
        int64_t s = 0;
        for (int j = -r; j <= r; ++j)
          for (int i = -r; i <= r; ++i)
            s += (int64_t)pix(L, pitch, W, H, x + i, y + j) * pix(R, pitch, W, H, x - d + i, y + j);
        S_RT[((ptrdiff_t)y * W + x) * D + d] = s;
      }
  return 0;
}

/* One element of the cross sum above. */
int64_t oracle_cross_sum_at(const uint8_t* L, const uint8_t* R, int pitch, int W, int H, int r, int x, int y, int d) {
  int64_t s = 0;
  for (int j = -r; j <= r; ++j)
    for (int i = -r; i <= r; ++i)
      s += (int64_t)pix(L, pitch, W, H, x + i, y + j) * pix(R, pitch, W, H, x - d + i, y + j);
  return s;
}

/* ---------------------------------------------------------------------------
 * ZNCC by its defining formula (Eq. ZNCC): deviations from the window means,
 * their cross sum over the standard deviations.  Returns z in [-1, 1].
 * Zero variance (exact integer test on l^2*sum(I^2) - (sum I)^2) gives z = 0.
 * ------------------------------------------------------------------------- */
double oracle_zncc_at(const uint8_t* L, const uint8_t* R, int pitch, int W, int H, int r, int x, int y,
                      int d) {
  const int l = 2 * r + 1;
  const double N = (double)l * l;
  int64_t sl = 0, sll = 0, st = 0, stt = 0;
  for (int j = -r; j <= r; ++j)
    for (int i = -r; i <= r; ++i) {
      int64_t a = pix(L, pitch, W, H, x + i, y + j);
      int64_t b = pix(R, pitch, W, H, x - d + i, y + j);
      sl += a;
      sll += a * a;
      st += b;
      stt += b * b;
    }
  const int64_t NL = (int64_t)l * l;
  if (NL * sll - sl * sl == 0 || NL * stt - st * st == 0) return 0.0;
  const double mean_r = (double)sl / N, mean_t = (double)st / N;
  double num = 0.0, var_r = 0.0, var_t = 0.0;
  for (int j = -r; j <= r; ++j)
    for (int i = -r; i <= r; ++i) {
      double dr = pix(L, pitch, W, H, x + i, y + j) - mean_r;
      double dt = pix(R, pitch, W, H, x - d + i, y + j) - mean_t;
      num += dr * dt;
      var_r += dr * dr;
      var_t += dt * dt;
    }
  double z = num / (sqrt(var_r) * sqrt(var_t));
  if (z > 1.0) z = 1.0;
  if (z < -1.0) z = -1.0;
  return z;
}

/* Matching cost 1 - ZNCC for one disparity slice d, array [H][W]. */
int oracle_zncc_cost_slice(const uint8_t* L, const uint8_t* R, int pitch, int W, int H, int r, int d,
                           double* cost_hw) {
  if (W < 1 || H < 1 || r < 0 || d < 0 || pitch < W) return -1;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x)
      cost_hw[(ptrdiff_t)y * W + x] = 1.0 - oracle_zncc_at(L, R, pitch, W, H, r, x, y, d);
  return 0;
}

/* Matching cost 1 - ZNCC for the whole volume, array [H][W][D]. */
int oracle_zncc_cost(const uint8_t* L, const uint8_t* R, int pitch, int W, int H, int D, int r,
                     double* cost_hwd) {
  if (W < 1 || H < 1 || D < 1 || r < 0 || pitch < W) return -1;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x)
      for (int d = 0; d < D; ++d)
        cost_hwd[((ptrdiff_t)y * W + x) * D + d] = 1.0 - oracle_zncc_at(L, R, pitch, W, H, r, x, y, d);
  return 0;
}

/* ---------------------------------------------------------------------------
 * DT edge weights (Eqs. k1-k4, a, weight):
 *   wh[y][x] = W_L(x,y) = exp(-1/sigma_s - |G(x,y) - G(x-1,y)| / (255 sigma_r)),  x >= 1
 *   wv[y][x] = W_U(x,y) = exp(-1/sigma_s - |G(x,y) - G(x,y-1)| / (255 sigma_r)),  y >= 1
 * wh[y][0] = wv[0][x] = 0 (no neighbour).  sigma_r = +inf disables the range term.
 * ------------------------------------------------------------------------- */
int oracle_dt_weights(const uint8_t* G, int pitch, int W, int H, double sigma_s, double sigma_r, double* wh,
                      double* wv) {
  if (W < 1 || H < 1 || !(sigma_s > 0.0) || !(sigma_r > 0.0) || pitch < W) return -1;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int g = G[(ptrdiff_t)y * pitch + x];
      double h = 0.0, v = 0.0;
      if (x >= 1) h = exp(-1.0 / sigma_s - fabs((double)(g - G[(ptrdiff_t)y * pitch + x - 1])) / (255.0 * sigma_r));
      if (y >= 1) v = exp(-1.0 / sigma_s - fabs((double)(g - G[(ptrdiff_t)(y - 1) * pitch + x])) / (255.0 * sigma_r));
      wh[(ptrdiff_t)y * W + x] = h;
      wv[(ptrdiff_t)y * W + x] = v;
    }
  return 0;
}

/* ---------------------------------------------------------------------------
 * DT recursions (Eqs. DT1-DT4), evaluated literally and in place on one
 * disparity slice whose element (x, y) sits at c[y*sy + x*sx]:
 *   L: C_L(x) = C(x)   + W_L(x) C_L(x-1)      x = 1 .. W-1
 *   R: C_R(x) = C_L(x) + W_R(x) C_R(x+1)      x = W-2 .. 0,  W_R(x) = wh(x+1)
 *   U: C_U(y) = C_R(y) + W_U(y) C_U(y-1)      y = 1 .. H-1
 *   D: C_D(y) = C_U(y) + W_D(y) C_D(y+1)      y = H-2 .. 0,  W_D(y) = wv(y+1)
 * repeated `iters` times; C is replaced by C_D after each sweep (Sec. III-B).
 * ------------------------------------------------------------------------- */
static void dt_slice_strided(double* c, ptrdiff_t sx, ptrdiff_t sy, int W, int H, const double* wh,
                             const double* wv, int iters) {
  for (int it = 0; it < iters; ++it) {
    for (int y = 0; y < H; ++y)
      for (int x = 1; x < W; ++x)
        c[y * sy + x * sx] += wh[(ptrdiff_t)y * W + x] * c[y * sy + (x - 1) * sx];
    for (int y = 0; y < H; ++y)
      for (int x = W - 2; x >= 0; --x)
        c[y * sy + x * sx] += wh[(ptrdiff_t)y * W + x + 1] * c[y * sy + (x + 1) * sx];
    for (int x = 0; x < W; ++x)
      for (int y = 1; y < H; ++y)
        c[y * sy + x * sx] += wv[(ptrdiff_t)y * W + x] * c[(y - 1) * sy + x * sx];
    for (int x = 0; x < W; ++x)
      for (int y = H - 2; y >= 0; --y)
        c[y * sy + x * sx] += wv[(ptrdiff_t)(y + 1) * W + x] * c[(y + 1) * sy + x * sx];
  }
}

/* One disparity slice, array [H][W], aggregated in place. */
int oracle_dt_slice(double* c_hw, int W, int H, const double* wh, const double* wv, int iters) {
  if (W < 1 || H < 1 || iters < 0) return -1;
  dt_slice_strided(c_hw, 1, W, W, H, wh, wv, iters);
  return 0;
}

/* Whole volume [H][W][D] aggregated in place, slice by slice. */
int oracle_dt_aggregate(double* vol_hwd, int W, int H, int D, const double* wh, const double* wv, int iters) {
  if (W < 1 || H < 1 || D < 1 || iters < 0) return -1;
  for (int d = 0; d < D; ++d) dt_slice_strided(vol_hwd + d, D, (ptrdiff_t)W * D, W, H, wh, wv, iters);
  return 0;
}

/* ---------------------------------------------------------------------------
 * WTA (Eq. WTA1): the smallest d attaining min_d C(x,y,d); vol is [H][W][D].
 * ------------------------------------------------------------------------- */
int oracle_wta(const double* vol_hwd, int W, int H, int D, int32_t* disp_hw) {
  if (W < 1 || H < 1 || D < 1) return -1;
  for (ptrdiff_t p = 0; p < (ptrdiff_t)W * H; ++p) {
    const double* c = vol_hwd + p * D;
    int best = 0;
    for (int d = 1; d < D; ++d)
      if (c[d] < c[best]) best = d;
    disp_hw[p] = best;
  }
  return 0;
}

/* ---------------------------------------------------------------------------
 * The whole path: cost 1 - ZNCC, DT with guide = reference (or target when
 * guide_target != 0), WTA.  cost_agg_hwd (nullable) receives the aggregated
 * volume; scratch is allocated here with malloc.
 * ------------------------------------------------------------------------- */
int oracle_stereo_solve(const uint8_t* L, const uint8_t* R, int pitch, int W, int H, int D, int r,
                        double sigma_s, double sigma_r, int iters, int guide_target, double* cost_agg_hwd,
                        int32_t* disp_hw) {
  if (W < 1 || H < 1 || D < 1 || r < 0 || iters < 0 || pitch < W) return -1;
  const size_t nv = (size_t)W * H * D, np = (size_t)W * H;
  double* vol = cost_agg_hwd ? cost_agg_hwd : (double*)malloc(nv * sizeof(double));
  double* wh = (double*)malloc(np * sizeof(double));
  double* wv = (double*)malloc(np * sizeof(double));
  int rc = -2;
  if (vol && wh && wv) {
    rc = oracle_zncc_cost(L, R, pitch, W, H, D, r, vol);
    if (rc == 0) rc = oracle_dt_weights(guide_target ? R : L, pitch, W, H, sigma_s, sigma_r, wh, wv);
    if (rc == 0) rc = oracle_dt_aggregate(vol, W, H, D, wh, wv, iters);
    if (rc == 0) rc = oracle_wta(vol, W, H, D, disp_hw);
  }
  free(wv);
  free(wh);
  if (!cost_agg_hwd) free(vol);
  return rc;
}

/* ---------------------------------------------------------------------------
 * 8-bit code of a normalised 16-bit cost (Sec. IV-C, data encoding and
 * decoding).  Only negative values carry information.  Of a negative value's
 * bits 14..0, six significant bits below its leading run of ones are kept,
 * with a 2-bit flag naming where they sit:
 *   flag 01: bits 14..9, when bits 14..11 are not all ones;
 *   flag 10: bits 10..5, when bits 14..11 are all ones but 10..7 are not;
 *   flag 11: bits 6..1,  when bits 14..7 are all ones.
 * The code is (six bits) << 2 | flag.  Reading for non-negative values: they
 * encode to the all-zero byte (taking the steps literally, 0 would get flag
 * 01 and decode to -32768).  Decoding: 0 gives 0; otherwise the six bits go
 * back to their position, every bit above them (through bit 15) is set and
 * every bit below is cleared.  A non-zero code with flag 00 is never produced
 * and decodes to 0.
 */
uint8_t oracle_i8_encode(int16_t v) {
  if (v >= 0) return 0;
  const unsigned u = (uint16_t)v;
  if (((u >> 11) & 0xFu) != 0xFu) return (uint8_t)((((u >> 9) & 0x3Fu) << 2) | 1u);
  if (((u >> 7) & 0xFu) != 0xFu) return (uint8_t)((((u >> 5) & 0x3Fu) << 2) | 2u);
  return (uint8_t)((((u >> 1) & 0x3Fu) << 2) | 3u);
}

int16_t oracle_i8_decode(uint8_t c) {
  const unsigned flag = c & 3u, six = c >> 2;
  if (c == 0 || flag == 0) return 0;
  const int pos = flag == 1 ? 9 : (flag == 2 ? 5 : 1); /* lowest bit of the six */
  const unsigned above = (0xFFFFu << (pos + 6)) & 0xFFFFu;
  return (int16_t)(uint16_t)(above | (six << pos));
}

/* ---------------------------------------------------------------------------
 * Single DT passes on one contiguous slice [H][W] (Eqs. DT1-DT4 one at a
 * time), and a run of them: passes first .. first+count-1 of the sequence
 * L, R, U, D, L, R, U, D, ... (pass k is L, R, U, D for k mod 4 = 0 .. 3).
 * count = 4*I from first = 0 is I sweeps, the same as oracle_dt_slice.
 * ------------------------------------------------------------------------- */
static void pass_l(double* c, int W, int H, const double* wh) {
  for (int y = 0; y < H; ++y)
    for (int x = 1; x < W; ++x) c[(ptrdiff_t)y * W + x] += wh[(ptrdiff_t)y * W + x] * c[(ptrdiff_t)y * W + x - 1];
}
static void pass_r(double* c, int W, int H, const double* wh) {
  for (int y = 0; y < H; ++y)
    for (int x = W - 2; x >= 0; --x)
      c[(ptrdiff_t)y * W + x] += wh[(ptrdiff_t)y * W + x + 1] * c[(ptrdiff_t)y * W + x + 1];
}
static void pass_u(double* c, int W, int H, const double* wv) {
  for (int x = 0; x < W; ++x)
    for (int y = 1; y < H; ++y) c[(ptrdiff_t)y * W + x] += wv[(ptrdiff_t)y * W + x] * c[(ptrdiff_t)(y - 1) * W + x];
}
static void pass_d(double* c, int W, int H, const double* wv) {
  for (int x = 0; x < W; ++x)
    for (int y = H - 2; y >= 0; --y)
      c[(ptrdiff_t)y * W + x] += wv[(ptrdiff_t)(y + 1) * W + x] * c[(ptrdiff_t)(y + 1) * W + x];
}
static void pass_k(double* c, int W, int H, const double* wh, const double* wv, int k) {
  switch (k & 3) {
    case 0: pass_l(c, W, H, wh); break;
    case 1: pass_r(c, W, H, wh); break;
    case 2: pass_u(c, W, H, wv); break;
    default: pass_d(c, W, H, wv); break;
  }
}

int oracle_dt_passes(double* c_hw, int W, int H, const double* wh, const double* wv, int first, int count) {
  if (W < 1 || H < 1 || first < 0 || count < 0) return -1;
  for (int k = first; k < first + count; ++k) pass_k(c_hw, W, H, wh, wv, k);
  return 0;
}

/* ---------------------------------------------------------------------------
 * The paper's narrow integer volumes (Sec. IV-C) as a whole path, in two
 * forms.  Common to both: a stored state v is kept as q = sat16(round(T v)),
 * rounding halves to even (T is the integer coefficient of Sec. IV-C, 21 in
 * Sec. V-C); a state stored as an 8-bit code keeps decode(encode(q)); a
 * stored state is read back as q / T.  The normalization of Eq. DT_new
 * subtracts, inside a pass, the pass input's value at d_arb = 0 at the same
 * pixel before the recursion, so the pass output's d_arb slice is zero.  The
 * DT's last pass is not stored: its output goes to the WTA as is.  Sweeps
 * after the first repeat the four passes (iters >= 1 only).
 *
 * form ORACLE_INT_PAPER -- the FastDT of Sec. V-C and Table II, one kernel per
 *   pass, so the volume is stored after every pass but the last (after L2R,
 *   R2L, U2D, and after D2U of every sweep but the last):
 *     Int16 (code8 = 0): every stored state is int16; the normalization runs
 *       in the U2D pass.
 *     Int8 (code8 = 1): the normalization runs in the R2L pass, whose output
 *       is stored as the 8-bit code ("encoding at the end of R2L"); U2D reads
 *       the decoded value ("decoding at the beginning of U2D"); the L2R and
 *       U2D outputs are int16.  Sweeps after the first are not in the paper;
 *       the D2U output that the next sweep reads is stored like R2L's, as the
 *       8-bit code.
 *   In later sweeps the d_arb slice entering the normalization is already
 *   zero, so subtracting it changes nothing; it is still done, as stated.
 * form ORACLE_INT_PAIRS -- the state crosses memory only between pass pairs:
 *   the raw cost is centred once, before the first pass (subtracting its
 *   d_arb = 0 slice; the passes are linear and keep a zero slice zero), and
 *   the output of every L,R pair and of every U,D pair but the last is
 *   stored, as int16 or (code8) as the 8-bit code.
 *
 * npasses in 1 .. 4*iters stops after that many passes (0: all of them); the
 * state returned is then the stored one when the stop is a store point.
 * final_hwd (nullable) receives that state; *saturated (nullable) counts the
 * stores whose rounded value fell outside the int16 range.  The WTA runs on
 * the returned state.
 * ------------------------------------------------------------------------- */
enum { ORACLE_INT_PAPER = 0, ORACLE_INT_PAIRS = 1 };

static double store_state(double v, double T, int code8, int64_t* sat) {
  double q = nearbyint(T * v); /* default rounding mode: to nearest, ties to even */
  if (q > 32767.0 || q < -32768.0) {
    ++*sat;
    q = q > 0.0 ? 32767.0 : -32768.0;
  }
  int16_t s = (int16_t)q;
  if (code8) s = oracle_i8_decode(oracle_i8_encode(s));
  return (double)s / T;
}

static void store_slice(double* c, size_t np, double T, int code8, int64_t* sat) {
  for (size_t p = 0; p < np; ++p) c[p] = store_state(c[p], T, code8, sat);
}

/* Eq. DT_new's subtraction: the pass input minus the input's d_arb slice.
 * With ref == NULL the slice being processed is the d_arb slice itself; its
 * input is first recorded into rec (if not NULL). */
static void normalize_slice(double* c, size_t np, const double* ref, double* rec) {
  if (rec) memcpy(rec, c, np * sizeof(double));
  for (size_t p = 0; p < np; ++p) c[p] -= ref ? ref[p] : c[p];
}

/* One disparity slice through the paper's per-pass form, npasses passes.
 * refs[it] is the d_arb slice's input to the normalizing pass of sweep it:
 * read when `record` is 0, written when it is 1 (the d_arb slice itself). */
static void int_slice_paper(double* c, int W, int H, const double* wh, const double* wv, int iters, int npasses,
                            double T, int code8, double* const* refs, int record, int64_t* sat) {
  const size_t np = (size_t)W * H;
  const int norm_pass = code8 ? 1 : 2; /* R2L for Int8, U2D for Int16 */
  for (int n = 0; n < npasses; ++n) {
    const int it = n / 4, k = n % 4;
    if (k == norm_pass) normalize_slice(c, np, record ? NULL : refs[it], record ? refs[it] : NULL);
    pass_k(c, W, H, wh, wv, k);
    if (n + 1 == 4 * iters) break; /* the DT's last pass feeds the WTA */
    store_slice(c, np, T, code8 && (k == 1 || k == 3), sat);
  }
}

/* One disparity slice through the pass-pair form (already centred): the
 * passes of the first npasses (a multiple of 2), storing after each pair but
 * the DT's last. */
static void int_slice_pairs(double* c, int W, int H, const double* wh, const double* wv, int iters, int npasses,
                            double T, int code8, int64_t* sat) {
  const size_t np = (size_t)W * H;
  for (int n = 0; n < npasses; n += 2) {
    pass_k(c, W, H, wh, wv, n % 4);
    pass_k(c, W, H, wh, wv, n % 4 + 1);
    if (n + 2 < 4 * iters) store_slice(c, np, T, code8, sat);
  }
}

int oracle_int_solve(const uint8_t* L, const uint8_t* R, int pitch, int W, int H, int D, int r, double sigma_s,
                     double sigma_r, int iters, int guide_target, double T, int code8, int form, int npasses,
                     double* final_hwd, int32_t* disp_hw, int64_t* saturated) {
  if (W < 1 || H < 1 || D < 1 || r < 0 || iters < 1 || pitch < W || !(T > 0.0)) return -1;
  if (form != ORACLE_INT_PAPER && form != ORACLE_INT_PAIRS) return -1;
  if (npasses == 0) npasses = 4 * iters;
  if (npasses < 1 || npasses > 4 * iters || (form == ORACLE_INT_PAIRS && npasses % 2)) return -1;
  const size_t np = (size_t)W * H;
  double* c0 = (double*)malloc(np * sizeof(double));
  double* c = (double*)malloc(np * sizeof(double));
  double* best = (double*)malloc(np * sizeof(double));
  double* wh = (double*)malloc(np * sizeof(double));
  double* wv = (double*)malloc(np * sizeof(double));
  double** refs = (double**)calloc((size_t)iters, sizeof(double*));
  int64_t sat = 0;
  int rc = -2, ok = c0 && c && best && wh && wv && refs;
  for (int it = 0; ok && it < iters; ++it) ok = (refs[it] = (double*)malloc(np * sizeof(double))) != NULL;
  if (ok) {
    rc = oracle_dt_weights(guide_target ? R : L, pitch, W, H, sigma_s, sigma_r, wh, wv);
    if (rc == 0) rc = oracle_zncc_cost_slice(L, R, pitch, W, H, r, 0, c0);
    for (int d = 0; rc == 0 && d < D; ++d) {
      rc = oracle_zncc_cost_slice(L, R, pitch, W, H, r, d, c);
      if (rc) break;
      if (form == ORACLE_INT_PAPER) {
        /* d = 0 (= d_arb) comes first and records its normalization inputs */
        int_slice_paper(c, W, H, wh, wv, iters, npasses, T, code8, refs, d == 0, &sat);
      } else {
        for (size_t p = 0; p < np; ++p) c[p] -= c0[p];
        int_slice_pairs(c, W, H, wh, wv, iters, npasses, T, code8, &sat);
      }
      for (size_t p = 0; p < np; ++p) {
        if (final_hwd) final_hwd[p * D + d] = c[p];
        if (d == 0 || c[p] < best[p]) { /* strict: the lowest d wins ties */
          best[p] = c[p];
          disp_hw[p] = d;
        }
      }
    }
  }
  if (saturated) *saturated = sat;
  for (int it = 0; refs && it < iters; ++it) free(refs[it]);
  free(refs);
  free(wv);
  free(wh);
  free(best);
  free(c);
  free(c0);
  return rc;
}

/* ---------------------------------------------------------------------------
 * Semi-global matching over four paths (the paper's system S1 combines its
 * ZNCC with SGM, P1 = 18 and P2 = 185 on costs multiplied by T, Sec. V-D).
 * Along a path r through pixels p_0, p_1, ...:
 *   L(p_0, d) = C(p_0, d)
 *   L(p_i, d) = C(p_i, d) + min( L(p_{i-1}, d),
 *                                L(p_{i-1}, d - 1) + P1, L(p_{i-1}, d + 1) + P1,
 *                                min_k L(p_{i-1}, k) + P2 ) - min_k L(p_{i-1}, k)
 * (terms with d - 1 < 0 or d + 1 >= D left out).  Paths: left to right,
 * right to left, top to bottom, bottom to top.  sum_hwd = the sum of the four
 * L, with C = scale * cost.  cost_hwd and sum_hwd are [H][W][D].
 */
static void sgm_path(const double* cost, double* sum, int W, int D, double p1, double p2, double scale,
                     const ptrdiff_t* pix, int n, double* prev, double* cur) {
  for (int i = 0; i < n; ++i) {
    const double* c = cost + pix[i] * D;
    double m = 0.0;
    if (i > 0) {
      m = prev[0];
      for (int k = 1; k < D; ++k) m = prev[k] < m ? prev[k] : m;
    }
    for (int d = 0; d < D; ++d) {
      double v = scale * c[d];
      if (i > 0) {
        double best = prev[d];
        if (d > 0 && prev[d - 1] + p1 < best) best = prev[d - 1] + p1;
        if (d + 1 < D && prev[d + 1] + p1 < best) best = prev[d + 1] + p1;
        if (m + p2 < best) best = m + p2;
        v += best - m;
      }
      cur[d] = v;
      sum[pix[i] * D + d] += v;
    }
    double* t = prev;
    prev = cur;
    cur = t;
  }
  (void)W;
}

int oracle_sgm_aggregate(const double* cost_hwd, int W, int H, int D, double p1, double p2, double scale,
                         double* sum_hwd) {
  if (W < 1 || H < 1 || D < 1 || !(p1 >= 0.0) || !(p2 >= p1)) return -1;
  const int n = W > H ? W : H;
  ptrdiff_t* pix = (ptrdiff_t*)malloc(sizeof(ptrdiff_t) * (size_t)n);
  double* a = (double*)malloc(sizeof(double) * (size_t)D);
  double* b = (double*)malloc(sizeof(double) * (size_t)D);
  if (!pix || !a || !b) {
    free(pix);
    free(a);
    free(b);
    return -2;
  }
  memset(sum_hwd, 0, sizeof(double) * (size_t)W * H * D);
  for (int y = 0; y < H; ++y) {
    for (int x = 0; x < W; ++x) pix[x] = (ptrdiff_t)y * W + x;  /* left to right */
    sgm_path(cost_hwd, sum_hwd, W, D, p1, p2, scale, pix, W, a, b);
    for (int x = 0; x < W; ++x) pix[x] = (ptrdiff_t)y * W + (W - 1 - x);  /* right to left */
    sgm_path(cost_hwd, sum_hwd, W, D, p1, p2, scale, pix, W, a, b);
  }
  for (int x = 0; x < W; ++x) {
    for (int y = 0; y < H; ++y) pix[y] = (ptrdiff_t)y * W + x;  /* top to bottom */
    sgm_path(cost_hwd, sum_hwd, W, D, p1, p2, scale, pix, H, a, b);
    for (int y = 0; y < H; ++y) pix[y] = (ptrdiff_t)(H - 1 - y) * W + x;  /* bottom to top */
    sgm_path(cost_hwd, sum_hwd, W, D, p1, p2, scale, pix, H, a, b);
  }
  free(pix);
  free(a);
  free(b);
  return 0;
}
