// zdt_lib.hip -- the C ABI declared in include/zdt.h.
//
// Validation, launch-shape selection and per-launch HIP-event timing.  The
// device work is in zdt_device.hpp; its compiled instances live in
// zdt_inst_<type>.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "zdt.h"
#include "zdt_host.hpp"

namespace zdt {

namespace {
thread_local std::string g_err;

struct ProfAcc {
  double ms = 0.0;
  int64_t n = 0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
std::vector<std::pair<std::string, ProfAcc>> g_prof_acc;
std::mutex g_kernel_mu;
struct KernelState {
  int rc = ZDT_OK;       // ZDT_OK, or why the kernel is refused
  size_t lds_limit = 0;  // dynamic LDS the kernel has been allowed above the 64 KB default
};
std::unordered_map<const void*, KernelState> g_kernel_ok;
}  // namespace

int prepare_kernel(const void* kernel, const char* name, size_t lds) {
  std::lock_guard<std::mutex> lk(g_kernel_mu);
  auto it = g_kernel_ok.find(kernel);
  if (it == g_kernel_ok.end()) {
    hipFuncAttributes attr{};
    const hipError_t e = hipFuncGetAttributes(&attr, kernel);
    if (e != hipSuccess) return fail(ZDT_EHIP, "%s: hipFuncGetAttributes: %s", name, hipGetErrorString(e));
    KernelState st{};
    if (attr.localSizeBytes > kMaxScratchBytes)
      st.rc = fail(ZDT_EUNSUPPORTED, "%s: kernel needs %zu B of scratch per lane (limit %d)", name,
                   (size_t)attr.localSizeBytes, kMaxScratchBytes);
    it = g_kernel_ok.emplace(kernel, st).first;
  }
  KernelState& st = it->second;
  if (st.rc != ZDT_OK) return fail(st.rc, "%s: kernel was refused (per-lane scratch too large)", name);
  if (lds > 65536 && lds > st.lds_limit) {
    const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return fail(ZDT_EHIP, "%s: cannot reserve %zu B of LDS: %s", name, lds, hipGetErrorString(e));
    st.lds_limit = lds;
  }
  return ZDT_OK;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

// Set while a call that must not allocate is enqueueing: no timing events then.
thread_local bool g_no_alloc = false;

bool prof_begin(ProfRec& rec, hipStream_t s) {
  if (g_no_alloc) return false;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return false;
  }
  rec.start = rec.stop = nullptr;
  if (hipEventCreate(&rec.start) != hipSuccess || hipEventCreate(&rec.stop) != hipSuccess ||
      hipEventRecord(rec.start, s) != hipSuccess) {
    if (rec.start) (void)hipEventDestroy(rec.start);
    if (rec.stop) (void)hipEventDestroy(rec.stop);
    rec.start = rec.stop = nullptr;
    return false;
  }
  return true;
}

void prof_end(ProfRec& rec, hipStream_t s) {
  if (hipEventRecord(rec.stop, s) != hipSuccess) {
    (void)hipEventDestroy(rec.start);
    (void)hipEventDestroy(rec.stop);
    return;
  }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_pending.push_back(rec);
}

}  // namespace zdt

using namespace zdt;

namespace {

// l = 2r + 1 <= 15: every window sum stays below 2^32 and each cost numerator
// l^2 S_RT - S_R S_T, whose magnitude is at most l^4 * 127.5^2 < 2^31, is exact
// when formed in wrapping 32-bit arithmetic.
constexpr int kMaxRadius = 7;

size_t dtype_size(int t) { return t == ZDT_F32 ? 4 : (t == ZDT_I8 ? 1 : 2); }
bool int_vol(int t) { return t == ZDT_I16 || t == ZDT_I8; }
// The paper's integer coefficient T (Sec. IV-C, T = 21 in its system).
constexpr float kIntScale = 21.0f;

int check_params(const zdt_params* p, const char* who) {
  if (!p) return fail(ZDT_EINVAL, "%s: params is NULL", who);
  if (p->width < 1 || p->height < 1) return fail(ZDT_EINVAL, "%s: width/height must be >= 1", who);
  if (p->pitch < p->width) return fail(ZDT_EINVAL, "%s: pitch %d < width %d", who, p->pitch, p->width);
  if (p->max_disp < 1) return fail(ZDT_EINVAL, "%s: max_disp must be >= 1", who);
  if (p->radius < 0) return fail(ZDT_EINVAL, "%s: radius must be >= 0", who);
  if (p->radius > kMaxRadius)
    return fail(ZDT_EUNSUPPORTED, "%s: radius %d > %d (32-bit exact sums need l <= 15)", who, p->radius, kMaxRadius);
  if (!(p->sigma_s > 0.0f) || std::isinf(p->sigma_s))
    return fail(ZDT_EINVAL, "%s: sigma_s must be finite and > 0", who);
  if (!(p->sigma_r > 0.0f)) return fail(ZDT_EINVAL, "%s: sigma_r must be > 0 (or +inf)", who);
  if (p->dt_iters < 0) return fail(ZDT_EINVAL, "%s: dt_iters must be >= 0", who);
  if (p->vol_dtype < ZDT_F32 || p->vol_dtype > ZDT_I8)
    return fail(ZDT_EINVAL, "%s: unknown vol_dtype %d", who, p->vol_dtype);
  if (p->flags & ~(ZDT_FLAG_NORMALIZE | ZDT_FLAG_GUIDE_TARGET))
    return fail(ZDT_EINVAL, "%s: unknown flags 0x%x", who, p->flags);
  for (int r : p->reserved)
    if (r != 0) return fail(ZDT_EINVAL, "%s: reserved fields must be zero", who);
  const long long nvol = (long long)p->width * p->height * p->max_disp;
  if (nvol >= (1LL << 31)) return fail(ZDT_EUNSUPPORTED, "%s: W*H*D = %lld exceeds 2^31-1 elements", who, nvol);
  if ((long long)nvol * (long long)dtype_size(p->vol_dtype) >= (1LL << 32))
    return fail(ZDT_EUNSUPPORTED, "%s: the volume must stay below 4 GiB (32-bit buffer offsets)", who);
  if (p->width > kMaxWaves * kHSegs64[kNumHSegs64 - 1] && !h_full_seg32(p->width))
    return fail(ZDT_EUNSUPPORTED, "%s: width %d > %d and not a multiple of 64 up to %d", who, p->width,
                kMaxWaves * kHSegs64[kNumHSegs64 - 1], 2 * kMaxWaves * kHSegs32[3]);
  if (p->height > kMaxWaves * kVSegs[kNumVSegs - 1])
    return fail(ZDT_EUNSUPPORTED, "%s: height %d > %d", who, p->height, kMaxWaves * kVSegs[kNumVSegs - 1]);
  return ZDT_OK;
}

// A line of n values split into segments of at most `seg` values: ceil(n/seg)
// segments of equal length segl (the last one shorter).
struct Split {
  int seg, segl, nseg;
};

Split split_with(int n, int seg) {
  const int n0 = (n + seg - 1) / seg;
  const int segl = (n + n0 - 1) / n0;
  return {seg, segl, (n + segl - 1) / segl};
}

// The smallest compiled segment length that splits n into <= maxseg segments.
Split split_line(int n, const int* segs, int nsegs, int maxseg) {
  for (int i = 0; i < nsegs; ++i)
    if (n <= maxseg * segs[i]) return split_with(n, segs[i]);
  return {0, 0, 0};
}

// Streamed H modes (sums, raw cost) take any segment length with 16 waves.
Split h_split_stream(const zdt_params* p) {
  const int segl = (p->width + kMaxWaves - 1) / kMaxWaves;
  return {0, segl, (p->width + segl - 1) / segl};
}

// ---- tile plans of the register-resident passes (zdt_plan in zdt.h)
struct Plan {
  int h_lanes, h_seg, v_lanes, v_seg;
};

bool in_list(int v, const int* list, int n) {
  for (int i = 0; i < n; ++i)
    if (list[i] == v) return true;
  return false;
}

bool h_plan_ok(int W, int lanes, int seg) {
  if (lanes == 32)
    return in_list(seg, kHSegs32, 4) && W % seg == 0 && (W / seg) % 2 == 0 && W / seg <= 2 * kMaxWaves;
  if (lanes == 64) return in_list(seg, kHSegs64, kNumHSegs64) && (W + seg - 1) / seg <= kMaxWaves;
  return false;
}

bool v_plan_ok(int H, int lanes, int seg) {
  if (lanes == 32)
    return in_list(seg, kVSegs32, kNumVSegs32) && H % seg == 0 && (H / seg) % 2 == 0 && H / seg <= 2 * kMaxWaves;
  if (lanes == 64) return in_list(seg, kVSegs, kNumVSegs) && (H + seg - 1) / seg <= kMaxWaves;
  return false;
}

Split h_split_plan(int W, const Plan& pl) {
  if (pl.h_lanes == 32) return {pl.h_seg, pl.h_seg, W / pl.h_seg};
  return split_with(W, pl.h_seg);
}

Split v_split_plan(int H, const Plan& pl) {
  if (pl.v_lanes == 32) return {pl.v_seg, pl.v_seg, H / pl.v_seg};
  return split_with(H, pl.v_seg);
}

// Default plan: two 32-lane segments per wave when the row splits into an even
// number of full segments (of the length h_default_seg32 picks), else 64-lane
// segments; the shortest 64-lane V
// segments that cover the column with 8 waves (measured faster than 16 shorter
// ones: fewer carries to compose, more workgroups per CU), else with up to 16
// waves -- except that the floating-point volumes then take two 32-lane
// segments per wave when the column splits into an even number of full ones:
// at 1080 rows two such workgroups share a CU where one 15-wave 64-lane
// workgroup fills it (1920x1080, D = 256: FP32 1.6 %, FP16 3.3 %, BF16 2.7 %
// faster per solve).  The integer volumes keep 64-lane segments (their 32-lane
// V kernels would need more than 64 VGPRs for two workgroups per CU).
Plan default_plan(const zdt_params* p) {
  Plan pl{};
  if (const int s32 = h_default_seg32(p->width)) {
    pl.h_lanes = 32;
    pl.h_seg = s32;
  } else {
    pl.h_lanes = 64;
    pl.h_seg = split_line(p->width, kHSegs64, kNumHSegs64, kMaxWaves).seg;
  }
  pl.v_lanes = 64;
  pl.v_seg = split_line(p->height, kVSegs, kNumVSegs, kMaxWaves / 2).seg;
  if (!pl.v_seg) {
    pl.v_seg = split_line(p->height, kVSegs, kNumVSegs, kMaxWaves).seg;
    if (!int_vol(p->vol_dtype))
      for (int seg : kVSegs32)
        if (v_plan_ok(p->height, 32, seg)) {
          pl.v_lanes = 32;
          pl.v_seg = seg;
          break;
        }
  }
  return pl;
}

// Every valid plan for the shape, the default first; H and V options that give
// the same split as a shorter compiled length are left out.
std::vector<Plan> plan_candidates(const zdt_params* p) {
  const int W = p->width, H = p->height;
  std::vector<std::pair<int, int>> hs;
  for (int seg : kHSegs32)
    if (h_plan_ok(W, 32, seg)) hs.push_back({32, seg});
  int last = -1;
  for (int seg : kHSegs64) {
    const int n0 = (W + seg - 1) / seg;
    if (h_plan_ok(W, 64, seg) && n0 != last) hs.push_back({64, seg});
    last = n0;
  }
  std::vector<std::pair<int, int>> vs;
  for (int seg : kVSegs32)
    if (v_plan_ok(H, 32, seg)) vs.push_back({32, seg});
  last = -1;
  for (int seg : kVSegs) {
    const int n0 = (H + seg - 1) / seg;
    if (v_plan_ok(H, 64, seg) && n0 != last) vs.push_back({64, seg});
    last = n0;
  }
  const Plan d = default_plan(p);
  std::vector<Plan> out{d};
  for (auto& h : hs)
    for (auto& v : vs)
      if (!(h.first == d.h_lanes && h.second == d.h_seg && v.first == d.v_lanes && v.second == d.v_seg))
        out.push_back({h.first, h.second, v.first, v.second});
  return out;
}

struct PlanKey {
  int W, H, D, R, dtype;
  bool operator<(const PlanKey& o) const {
    return std::tie(W, H, D, R, dtype) < std::tie(o.W, o.H, o.D, o.R, o.dtype);
  }
};
PlanKey plan_key(const zdt_params* p) { return {p->width, p->height, p->max_disp, p->radius, p->vol_dtype}; }

std::mutex g_plan_mu;
std::map<PlanKey, Plan> g_plans;  // plans pinned by zdt_set_plan / zdt_autotune

Plan plan_for(const zdt_params* p) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto it = g_plans.find(plan_key(p));
  return it != g_plans.end() ? it->second : default_plan(p);
}

bool normalized(const zdt_params* p) {
  return !int_vol(p->vol_dtype) && ((p->flags & ZDT_FLAG_NORMALIZE) || p->vol_dtype != ZDT_F32);
}

double one_minus_k(const zdt_params* p) { return -std::expm1(-1.0 / (double)p->sigma_s); }

// Scale applied after each pass pair (one pair = two passes of gain ~1/(1-K)).
float pair_scale(const zdt_params* p) {
  if (!normalized(p)) return 1.0f;
  const double omk = one_minus_k(p);
  return (float)(omk * omk);
}

double total_scale(const zdt_params* p) {
  if (!normalized(p)) return 1.0;
  return std::pow(one_minus_k(p), 4.0 * p->dt_iters);
}

float range_coef(const zdt_params* p) { return std::isinf(p->sigma_r) ? 0.0f : 1.0f / (255.0f * p->sigma_r); }

// Arguments shared by all jobs of a launch (pointers come from the job table).
HArgs make_hargs(const zdt_params* p, float out_scale) {
  HArgs a{};
  a.pitch = p->pitch;
  a.W = p->width;
  a.H = p->height;
  a.D = p->max_disp;
  a.inv_sigma_s = 1.0f / p->sigma_s;
  a.range_coef = range_coef(p);
  a.out_scale = out_scale;
  a.cost_scale = 1.0f;
  a.ref_role = kRefNone;
  return a;
}

VArgs make_vargs(const zdt_params* p, float out_scale) {
  VArgs a{};
  a.pitch = p->pitch;
  a.W = p->width;
  a.H = p->height;
  a.D = p->max_disp;
  a.inv_sigma_s = 1.0f / p->sigma_s;
  a.range_coef = range_coef(p);
  a.out_scale = out_scale;
  a.ref_sub = 0;
  return a;
}

// Launch an H-pass mode for n jobs.  `scaled` selects the exponent-scaled FP16
// working volume (tables carry the exponent maps).
int launch_h(const zdt_params* p, int dtype, int mode, bool scaled, HArgs a, const HJobs& t, int n, const Plan& pl,
             hipStream_t s) {
  int lps;
  Split sp;
  if (mode == kSums || mode == kCost) {
    lps = 64;
    sp = h_split_stream(p);
  } else {
    lps = pl.h_lanes;
    sp = h_split_plan(p->width, pl);
  }
  a.segl = sp.segl;
  a.nseg = sp.nseg;
  const int R = mode == kHPair ? 0 : p->radius;
  switch (dtype) {
    case ZDT_F32: return dispatch_h_f32(mode, R, sp.seg, lps, a, t, n, s);
    case ZDT_F16:
      return scaled ? dispatch_h_f16x(mode, R, sp.seg, lps, a, t, n, s) : dispatch_h_f16(mode, R, sp.seg, lps, a, t, n, s);
    case ZDT_BF16: return dispatch_h_bf16(mode, R, sp.seg, lps, a, t, n, s);
    case ZDT_I16: return dispatch_h_i16(mode, R, sp.seg, lps, a, t, n, s);
    case ZDT_I8: return dispatch_h_i8(mode, R, sp.seg, lps, a, t, n, s);
  }
  return fail(ZDT_EINVAL, "bad dtype %d", dtype);
}

int launch_v(const zdt_params* p, bool scaled, bool wta, VArgs a, const VJobs& t, int n, const Plan& pl,
             hipStream_t s) {
  const Split sp = v_split_plan(p->height, pl);
  a.segl = sp.segl;
  a.nseg = sp.nseg;
  const int lps = pl.v_lanes;
  switch (p->vol_dtype) {
    case ZDT_F32: return dispatch_v_f32(sp.seg, lps, wta, a, t, n, s);
    case ZDT_F16:
      return scaled ? dispatch_v_f16x(sp.seg, lps, wta, a, t, n, s) : dispatch_v_f16(sp.seg, lps, wta, a, t, n, s);
    case ZDT_BF16: return dispatch_v_bf16(sp.seg, lps, wta, a, t, n, s);
    case ZDT_I16: return dispatch_v_i16(sp.seg, lps, wta, a, t, n, s);
    case ZDT_I8: return dispatch_v_i8(sp.seg, lps, wta, a, t, n, s);
  }
  return fail(ZDT_EINVAL, "bad dtype %d", p->vol_dtype);
}

int dispatch_wta(int dtype, const void* vol, int npix, int D, int32_t* disp, hipStream_t s) {
  switch (dtype) {
    case ZDT_F32: return dispatch_wta_f32(vol, npix, D, disp, s);
    case ZDT_F16: return dispatch_wta_f16(vol, npix, D, disp, s);
    case ZDT_BF16: return dispatch_wta_bf16(vol, npix, D, disp, s);
    case ZDT_I16: return dispatch_wta_i16(vol, npix, D, disp, s);
    case ZDT_I8: return dispatch_wta_i8(vol, npix, D, disp, s);
  }
  return fail(ZDT_EINVAL, "bad dtype %d", dtype);
}

// Workspace of stereo_solve: for FP16 working volumes two gain maps (the
// H pairs write A, the V pairs write B), then the WTA partial minima of the
// disparity chunks (one V lane per disparity; chunks of 32 or 64 disparities
// depending on the plan, so the size covers 32).
struct WsLayout {
  size_t gain_a, gain_b, ref, part_val, part_idx, total;
};
size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }
int wta_chunks(const zdt_params* p, int v_lanes) { return (p->max_disp + v_lanes - 1) / v_lanes; }
WsLayout ws_layout(const zdt_params* p) {
  WsLayout L{};
  const size_t npix = (size_t)p->width * p->height;
  size_t o = 0;
  if (p->vol_dtype == ZDT_F16 && p->dt_iters > 0) {
    L.gain_a = o;
    o += align256(npix * sizeof(float));
    L.gain_b = o;
    o += align256(npix * sizeof(float));
  }
  if (int_vol(p->vol_dtype) && p->dt_iters > 0) {  // the d = 0 slice the first sweep normalizes by
    L.ref = o;
    o += align256(npix * sizeof(float));
  }
  if (p->dt_iters > 0 && wta_chunks(p, 32) > 1) {
    L.part_val = o;
    o += align256((size_t)wta_chunks(p, 32) * npix * sizeof(float));
    L.part_idx = o;
    o += align256((size_t)wta_chunks(p, 32) * npix * sizeof(int32_t));
  }
  L.total = o;
  return L;
}

// One pair's device buffers.
struct JobPtrs {
  const uint8_t* left;
  const uint8_t* right;
  int32_t* disp;
  void* vol;
  void* ws;
};

// stereo_solve for n <= kMaxJobs pairs that share every parameter: each stage
// is one launch over all of them (grid z = job).
int solve_group(const zdt_params* p, const JobPtrs* jobs, int n, hipStream_t s) {
  if (n < 1 || n > kMaxJobs) return fail(ZDT_EINVAL, "solve_group: %d jobs", n);
  const Plan pl = plan_for(p);
  const WsLayout L = ws_layout(p);
  const bool scaled = p->vol_dtype == ZDT_F16;  // gain-scaled FP16 working volume
  const bool ints = int_vol(p->vol_dtype);       // T-scaled integer volume (Sec. IV-C)
  const int vchunks = wta_chunks(p, pl.v_lanes);
  const bool multi = vchunks > 1;
  HJobs ht{};
  VJobs vt{};
  WJobs wt{};
  for (int i = 0; i < n; ++i) {
    const JobPtrs& j = jobs[i];
    const uint8_t* guide = (p->flags & ZDT_FLAG_GUIDE_TARGET) ? j.right : j.left;
    float* ga = scaled ? (float*)((char*)j.ws + L.gain_a) : nullptr;
    float* gb = scaled ? (float*)((char*)j.ws + L.gain_b) : nullptr;
    float* pv = multi ? (float*)((char*)j.ws + L.part_val) : nullptr;
    int32_t* pi = multi ? (int32_t*)((char*)j.ws + L.part_idx) : nullptr;
    float* rf = ints ? (float*)((char*)j.ws + L.ref) : nullptr;
    ht.j[i] = {j.left, j.right, guide, j.vol, gb, ga, rf};                    // H pairs: B -> A
    vt.j[i] = {guide, j.vol, ga, gb, multi ? nullptr : j.disp, pv, pi, rf};  // V pairs: A -> B
    wt.j[i] = {pv, pi, j.disp};
  }
  // An FP16 working volume is scaled per pixel by its gain and needs no
  // global scale; integer volumes hold T times the value (the fused pass
  // scales the raw cost); the other types take the (1-K)-per-pass
  // normalisation.
  const float sc = (scaled || ints) ? 1.0f : pair_scale(p);
  HArgs ha = make_hargs(p, sc);
  VArgs va = make_vargs(p, sc);
  if (ints) ha.cost_scale = kIntScale;
  int rc = ZDT_OK;
  // sweep 1: cost fused with L, R; then U, D.  Sweeps 2..I: L, R; U, D.  The
  // last U, D pair carries the WTA and writes no volume.  Integer volumes
  // follow the FastDT of Sec. V-C (see IntRef): the first sweep's Int8 R2L
  // subtracts the L2R output's d = 0 slice, taken by a reference launch over
  // disparity chunk 0; Int16's first U2D subtracts the R2L output's d = 0
  // slice, written by the fused pass.
  if (ints && p->vol_dtype == ZDT_I8) {
    HArgs hr = ha;
    hr.ref_role = kRefL2ROut;
    rc = launch_h(p, p->vol_dtype, kCostHPair, scaled, hr, ht, n, pl, s);
    ha.ref_role = kRefL2RIn;
  } else if (ints) {
    ha.ref_role = kRefR2LOut;
  }
  if (rc == ZDT_OK) rc = launch_h(p, p->vol_dtype, kCostHPair, scaled, ha, ht, n, pl, s);
  ha.ref_role = kRefNone;
  for (int it = 0; rc == ZDT_OK && it < p->dt_iters; ++it) {
    if (it > 0 && (rc = launch_h(p, p->vol_dtype, kHPair, scaled, ha, ht, n, pl, s))) break;
    va.ref_sub = (it == 0 && p->vol_dtype == ZDT_I16) ? 1 : 0;
    rc = launch_v(p, scaled, it + 1 == p->dt_iters, va, vt, n, pl, s);
  }
  if (rc == ZDT_OK && multi) {
    const dim3 grid((unsigned)((p->width + kCombineTile - 1) / kCombineTile),
                    (unsigned)((p->height + kCombineTile - 1) / kCombineTile), n);
    rc = launch("wta_combine", wta_combine_kernel, grid, dim3(kCombineTile * 8), 0, s, wt, vchunks, p->width,
                p->height);
  }
  return rc;
}

// The raw-cost path (dt_iters = 0): streamed cost volume, then the WTA.
int solve_raw(const zdt_params* p, const JobPtrs& j, hipStream_t s) {
  HJobs t{};
  t.j[0] = {j.left, j.right, nullptr, j.vol, nullptr, nullptr, nullptr};
  const Plan pl = plan_for(p);
  int rc = launch_h(p, p->vol_dtype, kCost, false, make_hargs(p, int_vol(p->vol_dtype) ? kIntScale : 1.0f), t, 1,
                    pl, s);
  if (rc) return rc;
  return dispatch_wta(p->vol_dtype, j.vol, p->width * p->height, p->max_disp, j.disp, s);
}

// Integer volumes keep every DT state but the last as a T-scaled int16.  The
// raw costs lie in [0, 2]; a pass with weights in [0, K] multiplies the largest
// magnitude by at most 1/(1-K); the normalization subtracts one non-negative
// state from another, which cannot grow it; a store adds at most 1/2.  A
// stored state can therefore leave the int16 range only if
//   s_n = s_{n-1} / (1-K) + 1/2,  s_0 = 2 T,
// exceeds 32767 for some n < 4 I (the DT's last pass is not stored).  Such
// parameters are refused rather than saturated silently.
int check_int_range(const zdt_params* p, const char* who) {
  if (!int_vol(p->vol_dtype) || p->dt_iters < 1) return ZDT_OK;
  const double g = 1.0 / one_minus_k(p);
  double b = 2.0 * kIntScale;
  for (int n = 1; n < 4 * p->dt_iters; ++n) {
    b = b * g + 0.5;
    if (b > 32767.0)
      return fail(ZDT_EUNSUPPORTED,
                  "%s: with sigma_s = %g and %d sweeps a stored int16 state could reach %.4g after %d passes "
                  "(T = %g); integer volumes need that bound below 32767", who, p->sigma_s, p->dt_iters, b, n,
                  (double)kIntScale);
  }
  return ZDT_OK;
}

int check_job(const zdt_params* p, const uint8_t* left, const uint8_t* right, const int32_t* disp, const void* vol,
              const void* ws, const char* who) {
  int rc = check_params(p, who);
  if (rc) return rc;
  if ((rc = check_int_range(p, who))) return rc;
  if (!left || !right || !disp || !vol) return fail(ZDT_EINVAL, "%s: NULL image, disparity or volume pointer", who);
  if (p->vol_dtype == ZDT_I8 && p->dt_iters == 0)
    return fail(ZDT_EUNSUPPORTED, "%s: 8-bit coded volumes need dt_iters >= 1 (raw costs code to zero)", who);
  if (p->dt_iters > 0) {
    const size_t need = ws_layout(p).total;
    if (need && !ws) return fail(ZDT_EINVAL, "%s: a workspace of %zu B is required", who, need);
  }
  return ZDT_OK;
}

zdt_plan to_c(const Plan& pl) { return zdt_plan{pl.h_lanes, pl.h_seg, pl.v_lanes, pl.v_seg}; }

// ---- the workspace of stereo_solve_static_ws: an array in the library's code
// object, so every GPU that loads the library holds its own copy until the
// process ends.  In host code `scratch` only names the symbol; its device
// address (one per GPU) is looked up once per device and kept here.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) uint8_t scratch[ZDT_STATIC_WS_BYTES];

namespace {
// Device address of `scratch` on the GPU that `stream` belongs to (the
// current GPU for the NULL stream).
int scratch_for(hipStream_t stream, void** out, const char* who) {
  int cur = -1, dev = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(ZDT_EHIP, "%s: hipGetDevice failed", who);
  dev = cur;
  if (stream && hipStreamGetDevice(stream, &dev) != hipSuccess)
    return fail(ZDT_EHIP, "%s: hipStreamGetDevice failed", who);
  if (dev < 0 || dev >= kMaxDevices) return fail(ZDT_EUNSUPPORTED, "%s: device %d", who, dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    if (dev != cur && hipSetDevice(dev) != hipSuccess) return fail(ZDT_EHIP, "%s: hipSetDevice(%d) failed", who, dev);
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (dev != cur) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr)
      return fail(ZDT_EHIP, "%s: hipGetSymbolAddress(scratch) on device %d: %s", who, dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return ZDT_OK;
}

// Plan cache file: one line per shape,
//   zdt-plan W H D R dtype : h_lanes h_seg v_lanes v_seg  (best_us)
bool read_cached_plan(const char* path, const zdt_params* p, Plan* out) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[256];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    int W, H, D, R, dt, hl, hs, vl, vs;
    if (std::sscanf(line, "zdt-plan %d %d %d %d %d : %d %d %d %d", &W, &H, &D, &R, &dt, &hl, &hs, &vl, &vs) == 9 &&
        W == p->width && H == p->height && D == p->max_disp && R == p->radius && dt == p->vol_dtype &&
        h_plan_ok(W, hl, hs) && v_plan_ok(H, vl, vs)) {
      *out = {hl, hs, vl, vs};
      found = true;  // the last matching line wins
    }
  }
  std::fclose(f);
  return found;
}
}  // namespace

// =================================================================== C ABI
extern "C" {

const char* zdt_last_error(void) { return g_err.c_str(); }

size_t zdt_volume_size(const zdt_params* p) {
  if (check_params(p, "zdt_volume_size") != ZDT_OK) return 0;
  return (size_t)p->width * p->height * p->max_disp * dtype_size(p->vol_dtype);
}

size_t zdt_workspace_size(const zdt_params* p) {
  if (check_params(p, "zdt_workspace_size") != ZDT_OK) return 0;
  const WsLayout L = ws_layout(p);
  return L.total;
}

int zncc_cost_volume(const zdt_params* p, const uint8_t* left, const uint8_t* right, void* cost, void* stream) {
  int rc = check_params(p, "zncc_cost_volume");
  if (rc) return rc;
  if (!left || !right || !cost) return fail(ZDT_EINVAL, "zncc_cost_volume: NULL image or volume pointer");
  HJobs t{};
  if (p->vol_dtype == ZDT_I8)
    return fail(ZDT_EUNSUPPORTED, "zncc_cost_volume: raw costs are non-negative, their 8-bit codes are all zero");
  t.j[0] = {left, right, nullptr, cost, nullptr, nullptr, nullptr};
  const float sc = int_vol(p->vol_dtype) ? kIntScale : 1.0f;
  return launch_h(p, p->vol_dtype, kCost, false, make_hargs(p, sc), t, 1, plan_for(p), (hipStream_t)stream);
}

int zncc_window_sums(const zdt_params* p, const uint8_t* left, const uint8_t* right, int32_t* s_l, int32_t* s_ll,
                     int32_t* s_t, int32_t* s_tt, int32_t* s_rt, void* stream) {
  int rc = check_params(p, "zncc_window_sums");
  if (rc) return rc;
  if (!left || !right) return fail(ZDT_EINVAL, "zncc_window_sums: NULL image pointer");
  HArgs a = make_hargs(p, 1.0f);
  a.s_rt = s_rt;
  a.s_l = s_l;
  a.s_ll = s_ll;
  a.s_t = s_t;
  a.s_tt = s_tt;
  HJobs t{};
  t.j[0] = {left, right, nullptr, nullptr, nullptr, nullptr, nullptr};
  return launch_h(p, ZDT_F32, kSums, false, a, t, 1, plan_for(p), (hipStream_t)stream);
}

size_t zdt_integral_workspace_size(const zdt_params* p) {
  if (check_params(p, "zdt_integral_workspace_size") != ZDT_OK) return 0;
  size_t words = 0;
  for (int im = 0; im < 2; ++im) words += 2 * integral_words(p->width, p->height, p->max_disp, p->radius, im);
  return words * 4;
}

int zncc_window_sums_integral(const zdt_params* p, const uint8_t* left, const uint8_t* right, int32_t* s_l,
                              int32_t* s_ll, int32_t* s_t, int32_t* s_tt, void* ws, void* stream) {
  int rc = check_params(p, "zncc_window_sums_integral");
  if (rc) return rc;
  if (!left || !right) return fail(ZDT_EINVAL, "zncc_window_sums_integral: NULL image pointer");
  if (!ws) return fail(ZDT_EINVAL, "zncc_window_sums_integral: NULL workspace");
  if ((uintptr_t)ws & 3) return fail(ZDT_EINVAL, "zncc_window_sums_integral: workspace must be 4-byte aligned");
  return integral_window_sums(left, right, p->pitch, p->width, p->height, p->max_disp, p->radius, s_l, s_ll, s_t,
                              s_tt, ws, (hipStream_t)stream);
}

int dt_aggregate(const zdt_params* p, const uint8_t* guide, void* cost, double* applied_scale, void* stream) {
  int rc = check_params(p, "dt_aggregate");
  if (rc) return rc;
  if (!guide || !cost) return fail(ZDT_EINVAL, "dt_aggregate: NULL guide or volume pointer");
  if (int_vol(p->vol_dtype))
    return fail(ZDT_EUNSUPPORTED, "dt_aggregate: integer volumes are produced only inside stereo_solve");
  hipStream_t s = (hipStream_t)stream;
  const float sc = pair_scale(p);
  const Plan pl = plan_for(p);
  HJobs ht{};
  ht.j[0] = {nullptr, nullptr, guide, cost, nullptr, nullptr, nullptr};
  VJobs vt{};
  vt.j[0] = {guide, cost, nullptr, nullptr, nullptr, nullptr, nullptr};
  for (int it = 0; it < p->dt_iters; ++it) {
    if ((rc = launch_h(p, p->vol_dtype, kHPair, false, make_hargs(p, sc), ht, 1, pl, s))) return rc;
    if ((rc = launch_v(p, false, false, make_vargs(p, sc), vt, 1, pl, s))) return rc;
  }
  if (applied_scale) *applied_scale = total_scale(p);
  return ZDT_OK;
}

int wta_disparity(const zdt_params* p, const void* cost, int32_t* disp, void* stream) {
  int rc = check_params(p, "wta_disparity");
  if (rc) return rc;
  if (!cost || !disp) return fail(ZDT_EINVAL, "wta_disparity: NULL volume or disparity pointer");
  return dispatch_wta(p->vol_dtype, cost, p->width * p->height, p->max_disp, disp, (hipStream_t)stream);
}

int stereo_solve(const zdt_params* p, const uint8_t* left, const uint8_t* right, int32_t* disp, void* vol, void* ws,
                 void* stream) {
  int rc = check_job(p, left, right, disp, vol, ws, "stereo_solve");
  if (rc) return rc;
  const JobPtrs j{left, right, disp, vol, ws};
  if (p->dt_iters == 0) return solve_raw(p, j, (hipStream_t)stream);
  return solve_group(p, &j, 1, (hipStream_t)stream);
}

int stereo_solve_static_ws(const zdt_params* p, const uint8_t* left, const uint8_t* right, int32_t* disp, void* vol,
                           void* stream) {
  int rc = check_params(p, "stereo_solve_static_ws");
  if (rc) return rc;
  const size_t need = p->dt_iters > 0 ? ws_layout(p).total : 0;
  if (need > ZDT_STATIC_WS_BYTES)
    return fail(ZDT_EUNSUPPORTED, "stereo_solve_static_ws: the parameters need %zu B of workspace, more than the %u B "
                "the library holds", need, (unsigned)ZDT_STATIC_WS_BYTES);
  hipStream_t s = (hipStream_t)stream;
  void* ws = nullptr;
  if (need && (rc = scratch_for(s, &ws, "stereo_solve_static_ws"))) return rc;
  if ((rc = check_job(p, left, right, disp, vol, ws, "stereo_solve_static_ws"))) return rc;
  const JobPtrs j{left, right, disp, vol, ws};
  g_no_alloc = true;
  rc = p->dt_iters == 0 ? solve_raw(p, j, s) : solve_group(p, &j, 1, s);
  g_no_alloc = false;
  return rc;
}

}  // extern "C"

namespace {
// ---- concurrent batches: two library-owned streams per GPU
// A batch is dealt over two streams forked from and joined back to the
// caller's stream, so the pairs' kernels share the GPU: one pair's cost and
// recursion launches fill the CUs while another's drain, and stages bound by
// arithmetic run beside stages bound by memory.  The streams (default
// priority, non-blocking) and events live until the process ends.
constexpr int kSideStreams = 2;
struct SideStreams {
  hipStream_t s[kSideStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kSideStreams] = {};
  std::mutex mu;  // one batch at a time enqueues on a GPU's pair of streams
};
SideStreams g_side[kMaxDevices];
std::mutex g_side_init_mu;

int side_streams_for(hipStream_t stream, SideStreams** out, const char* who) {
  int cur = -1, dev = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(ZDT_EHIP, "%s: hipGetDevice failed", who);
  dev = cur;
  if (stream && hipStreamGetDevice(stream, &dev) != hipSuccess)
    return fail(ZDT_EHIP, "%s: hipStreamGetDevice failed", who);
  if (dev < 0 || dev >= kMaxDevices) return fail(ZDT_EUNSUPPORTED, "%s: device %d", who, dev);
  std::lock_guard<std::mutex> lk(g_side_init_mu);
  SideStreams& ss = g_side[dev];
  if (!ss.fork) {
    if (dev != cur && hipSetDevice(dev) != hipSuccess) return fail(ZDT_EHIP, "%s: hipSetDevice(%d) failed", who, dev);
    bool ok = true;
    for (int k = 0; k < kSideStreams && ok; ++k)
      ok = (ss.s[k] || hipStreamCreateWithFlags(&ss.s[k], hipStreamNonBlocking) == hipSuccess) &&
           (ss.join[k] || hipEventCreateWithFlags(&ss.join[k], hipEventDisableTiming) == hipSuccess);
    // the fork event is made last: its presence marks the set complete
    if (ok) ok = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming) == hipSuccess;
    if (dev != cur) (void)hipSetDevice(cur);
    if (!ok) return fail(ZDT_EHIP, "%s: creating the batch streams on device %d failed", who, dev);
  }
  *out = &ss;
  return ZDT_OK;
}

int solve_one(const zdt_job& j, hipStream_t s) {
  const JobPtrs p{j.left, j.right, j.disp, j.vol, j.ws};
  return j.params.dt_iters == 0 ? solve_raw(&j.params, p, s) : solve_group(&j.params, &p, 1, s);
}

// Jobs with identical parameters share each stage's launch (up to kMaxJobs per
// grid), in submission order, all on `s`.
int solve_grouped(const zdt_job* jobs, int n, hipStream_t s) {
  std::vector<char> done(n, 0);
  std::vector<JobPtrs> group;
  for (int i = 0; i < n; ++i) {
    if (done[i]) continue;
    const zdt_params& p = jobs[i].params;
    group.clear();
    for (int k = i; k < n; ++k) {
      if (done[k] || std::memcmp(&jobs[k].params, &p, sizeof p) != 0) continue;
      done[k] = 1;
      group.push_back({jobs[k].left, jobs[k].right, jobs[k].disp, jobs[k].vol, jobs[k].ws});
    }
    for (size_t g0 = 0; g0 < group.size(); g0 += kMaxJobs) {
      const int m = (int)std::min<size_t>(kMaxJobs, group.size() - g0);
      int rc = ZDT_OK;
      if (p.dt_iters == 0) {
        for (int k = 0; k < m && rc == ZDT_OK; ++k) rc = solve_raw(&p, group[g0 + k], s);
      } else {
        rc = solve_group(&p, group.data() + g0, m, s);
      }
      if (rc) return rc;
    }
  }
  return ZDT_OK;
}

// Largest job first, each to the side stream with less work queued so far
// (work: cost values times the passes over them).
int solve_concurrent(const zdt_job* jobs, int n, hipStream_t s, SideStreams& ss) {
  std::vector<int> order(n);
  std::vector<double> work(n);
  for (int i = 0; i < n; ++i) {
    const zdt_params& p = jobs[i].params;
    order[i] = i;
    work[i] = (double)p.width * p.height * p.max_disp * (1 + 2 * p.dt_iters);
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  if (hipEventRecord(ss.fork, s) != hipSuccess) return fail(ZDT_EHIP, "stereo_solve_batch: hipEventRecord failed");
  for (int k = 0; k < kSideStreams; ++k)
    if (hipStreamWaitEvent(ss.s[k], ss.fork, 0) != hipSuccess)
      return fail(ZDT_EHIP, "stereo_solve_batch: hipStreamWaitEvent failed");
  double queued[kSideStreams] = {};
  int rc = ZDT_OK;
  for (int i : order) {
    int k = 0;
    for (int q = 1; q < kSideStreams; ++q)
      if (queued[q] < queued[k]) k = q;
    queued[k] += work[i];
    if ((rc = solve_one(jobs[i], ss.s[k]))) break;
  }
  // join even after an error, so that later work on `s` stays ordered after
  // whatever was enqueued
  for (int k = 0; k < kSideStreams; ++k)
    if (hipEventRecord(ss.join[k], ss.s[k]) != hipSuccess || hipStreamWaitEvent(s, ss.join[k], 0) != hipSuccess)
      if (rc == ZDT_OK) rc = fail(ZDT_EHIP, "stereo_solve_batch: joining the batch streams failed");
  return rc;
}
}  // namespace

extern "C" {

int stereo_solve_batch(const zdt_job* jobs, int32_t n, void* stream) {
  if (n < 0 || (n > 0 && !jobs)) return fail(ZDT_EINVAL, "stereo_solve_batch: %d jobs at %p", n, (const void*)jobs);
  for (int i = 0; i < n; ++i) {
    const zdt_job& j = jobs[i];
    int rc = check_job(&j.params, j.left, j.right, j.disp, j.vol, j.ws, "stereo_solve_batch");
    if (rc) return fail(rc, "stereo_solve_batch: job %d: %s", i, zdt_last_error());
  }
  hipStream_t s = (hipStream_t)stream;
  if (n < 2) return n == 1 ? solve_one(jobs[0], s) : ZDT_OK;
  // Under graph capture (and in the no-allocation path) the batch stays on
  // the caller's stream: grouped launches, no library streams in the graph.
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return fail(ZDT_EHIP, "stereo_solve_batch: hipStreamIsCapturing failed");
  if (g_no_alloc || cs != hipStreamCaptureStatusNone) return solve_grouped(jobs, n, s);
  SideStreams* ss = nullptr;
  int rc = side_streams_for(s, &ss, "stereo_solve_batch");
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(ss->mu);
  return solve_concurrent(jobs, n, s, *ss);
}

namespace {
// Shared checks of the SGM entry points: an FP32 or FP16 cost volume, an FP32
// sum volume, both 16-byte aligned and disjoint, D <= 256 (four disparities per
// lane), 0 <= P1 <= P2 and a finite non-negative cost scale.
int check_sgm(const zdt_params* p, const void* cost, const float* sum, float p1, float p2, float scale,
              const char* who) {
  int rc = check_params(p, who);
  if (rc) return rc;
  if (p->vol_dtype != ZDT_F32 && p->vol_dtype != ZDT_F16)
    return fail(ZDT_EUNSUPPORTED, "%s: SGM cost volumes are FP32 or FP16 (vol_dtype 0 or 1)", who);
  if (p->max_disp > 4 * kWave) return fail(ZDT_EUNSUPPORTED, "%s: max_disp %d > %d", who, p->max_disp, 4 * kWave);
  if (!(p1 >= 0.0f) || !(p2 >= p1) || std::isinf(p2))
    return fail(ZDT_EINVAL, "%s: penalties need 0 <= P1 <= P2 < inf (got %g, %g)", who, p1, p2);
  if (!(scale >= 0.0f) || std::isinf(scale)) return fail(ZDT_EINVAL, "%s: cost scale must be finite, >= 0", who);
  if (!cost || !sum) return fail(ZDT_EINVAL, "%s: NULL cost or sum volume", who);
  if (((uintptr_t)cost | (uintptr_t)sum) & 15) return fail(ZDT_EINVAL, "%s: volumes must be 16-byte aligned", who);
  const size_t n = (size_t)p->width * p->height * p->max_disp;
  const char *c = (const char*)cost, *q = (const char*)sum;
  if (c < q + n * 4 && q < c + n * dtype_size(p->vol_dtype))
    return fail(ZDT_EINVAL, "%s: the cost and sum volumes overlap", who);
  return ZDT_OK;
}

SgmArgs sgm_args(const zdt_params* p, const void* cost, float* sum, int32_t* disp, float p1, float p2, float scale) {
  return SgmArgs{cost, p->vol_dtype == ZDT_F16, sum, disp, p->width, p->height, p->max_disp, p1, p2, scale};
}
}  // namespace

int sgm_aggregate(const zdt_params* p, const void* cost, float* sum, float p1, float p2, float cost_scale,
                  void* stream) {
  int rc = check_sgm(p, cost, sum, p1, p2, cost_scale, "sgm_aggregate");
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const SgmArgs a = sgm_args(p, cost, sum, nullptr, p1, p2, cost_scale);
  if ((rc = dispatch_sgm(a, false, false, s))) return rc;
  return dispatch_sgm(a, true, false, s);
}

int sgm_disparity(const zdt_params* p, const void* cost, float* sum, int32_t* disp, float p1, float p2,
                  float cost_scale, void* stream) {
  int rc = check_sgm(p, cost, sum, p1, p2, cost_scale, "sgm_disparity");
  if (rc) return rc;
  if (!disp) return fail(ZDT_EINVAL, "sgm_disparity: NULL disparity pointer");
  hipStream_t s = (hipStream_t)stream;
  const SgmArgs a = sgm_args(p, cost, sum, disp, p1, p2, cost_scale);
  if ((rc = dispatch_sgm(a, false, false, s))) return rc;
  return dispatch_sgm(a, true, true, s);
}

int stereo_solve_sgm(const zdt_params* p, const uint8_t* left, const uint8_t* right, int32_t* disp, void* cost,
                     float* sum, float p1, float p2, float cost_scale, void* stream) {
  int rc = check_sgm(p, cost, sum, p1, p2, cost_scale, "stereo_solve_sgm");
  if (rc) return rc;
  if (!left || !right || !disp) return fail(ZDT_EINVAL, "stereo_solve_sgm: NULL image or disparity pointer");
  if ((rc = zncc_cost_volume(p, left, right, cost, stream))) return rc;
  return sgm_disparity(p, cost, sum, disp, p1, p2, cost_scale, stream);
}

// ---- graphs: stereo_solve_batch captured once, replayed many times
}  // extern "C"
struct zdt_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};
extern "C" {

int zdt_graph_create(const zdt_job* jobs, int32_t n, void* stream, zdt_graph** out) {
  if (!out) return fail(ZDT_EINVAL, "zdt_graph_create: NULL output");
  *out = nullptr;
  if (n < 1 || !jobs) return fail(ZDT_EINVAL, "zdt_graph_create: %d jobs at %p", n, (const void*)jobs);
  hipStream_t s = (hipStream_t)stream;
  if (!s) return fail(ZDT_EINVAL, "zdt_graph_create: capture needs a stream other than the NULL stream");
  // A first, eager run prepares every kernel (attribute queries, LDS limits)
  // so that the capture itself only records launches.
  int rc = stereo_solve_batch(jobs, n, stream);
  if (rc) return rc;
  zdt_graph* g = new (std::nothrow) zdt_graph();
  if (!g) return fail(ZDT_ENOMEM, "zdt_graph_create: out of host memory");
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    delete g;
    return fail(ZDT_EHIP, "zdt_graph_create: hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  g_no_alloc = true;  // no timing events inside the graph
  rc = stereo_solve_batch(jobs, n, stream);
  g_no_alloc = false;
  e = hipStreamEndCapture(s, &g->graph);
  if (rc == ZDT_OK && e != hipSuccess) rc = fail(ZDT_EHIP, "zdt_graph_create: hipStreamEndCapture: %s", hipGetErrorString(e));
  if (rc == ZDT_OK && (e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess)
    rc = fail(ZDT_EHIP, "zdt_graph_create: hipGraphInstantiate: %s", hipGetErrorString(e));
  if (rc) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return rc;
  }
  *out = g;
  return ZDT_OK;
}

int zdt_graph_launch(zdt_graph* g, void* stream) {
  if (!g || !g->exec) return fail(ZDT_EINVAL, "zdt_graph_launch: NULL graph");
  const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(ZDT_EHIP, "zdt_graph_launch: %s", hipGetErrorString(e));
  return ZDT_OK;
}

int zdt_graph_destroy(zdt_graph* g) {
  if (!g) return ZDT_OK;
  int rc = ZDT_OK;
  if (g->exec && hipGraphExecDestroy(g->exec) != hipSuccess) rc = fail(ZDT_EHIP, "zdt_graph_destroy: exec");
  if (g->graph && hipGraphDestroy(g->graph) != hipSuccess) rc = fail(ZDT_EHIP, "zdt_graph_destroy: graph");
  delete g;
  return rc;
}

int zdt_plan_candidates(const zdt_params* p, zdt_plan* out, int max) {
  int rc = check_params(p, "zdt_plan_candidates");
  if (rc) return rc;
  if (max < 0 || (max > 0 && !out)) return fail(ZDT_EINVAL, "zdt_plan_candidates: bad output array");
  const std::vector<Plan> c = plan_candidates(p);
  for (int i = 0; i < max && i < (int)c.size(); ++i) out[i] = to_c(c[i]);
  return (int)c.size();
}

int zdt_get_plan(const zdt_params* p, zdt_plan* out) {
  int rc = check_params(p, "zdt_get_plan");
  if (rc) return rc;
  if (!out) return fail(ZDT_EINVAL, "zdt_get_plan: NULL output");
  *out = to_c(plan_for(p));
  return ZDT_OK;
}

int zdt_set_plan(const zdt_params* p, const zdt_plan* plan) {
  int rc = check_params(p, "zdt_set_plan");
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  if (!plan) {
    g_plans.erase(plan_key(p));
    return ZDT_OK;
  }
  if (!h_plan_ok(p->width, plan->h_lanes, plan->h_seg) || !v_plan_ok(p->height, plan->v_lanes, plan->v_seg))
    return fail(ZDT_EINVAL, "zdt_set_plan: plan (%d, %d, %d, %d) does not fit %dx%d", plan->h_lanes, plan->h_seg,
                plan->v_lanes, plan->v_seg, p->width, p->height);
  g_plans[plan_key(p)] = {plan->h_lanes, plan->h_seg, plan->v_lanes, plan->v_seg};
  return ZDT_OK;
}

int zdt_autotune(const zdt_params* p, const char* cache_path, zdt_plan* chosen, void* stream) {
  int rc = check_params(p, "zdt_autotune");
  if (rc) return rc;
  Plan best{};
  if (cache_path && read_cached_plan(cache_path, p, &best)) {
    const zdt_plan c = to_c(best);
    if ((rc = zdt_set_plan(p, &c))) return rc;
    if (chosen) *chosen = c;
    return ZDT_OK;
  }
  if (p->dt_iters == 0) {  // nothing register-resident to tune
    if (chosen) *chosen = to_c(plan_for(p));
    return ZDT_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t img = (size_t)p->pitch * p->height, npix = (size_t)p->width * p->height;
  const size_t vbytes = npix * p->max_disp * dtype_size(p->vol_dtype), wbytes = ws_layout(p).total;
  uint8_t *left = nullptr, *right = nullptr;
  int32_t* disp = nullptr;
  void *vol = nullptr, *ws = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    (void)hipFree(left);
    (void)hipFree(right);
    (void)hipFree(disp);
    (void)hipFree(vol);
    (void)hipFree(ws);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc((void**)&left, img) != hipSuccess || hipMalloc((void**)&right, img) != hipSuccess ||
      hipMalloc((void**)&disp, npix * 4) != hipSuccess || hipMalloc(&vol, vbytes) != hipSuccess ||
      (wbytes && hipMalloc(&ws, wbytes) != hipSuccess) || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    release();
    return fail(ZDT_EHIP, "zdt_autotune: cannot allocate the %zu B trial buffers", 2 * img + npix * 4 + vbytes + wbytes);
  }
  {  // a textured trial pair (timings do not depend on the values)
    std::vector<uint8_t> h(img);
    uint32_t x = 12345u;
    for (auto& v : h) v = (uint8_t)((x = x * 1664525u + 1013904223u) >> 24);
    if (hipMemcpy(left, h.data(), img, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(right, h.data(), img, hipMemcpyHostToDevice) != hipSuccess) {
      release();
      return fail(ZDT_EHIP, "zdt_autotune: cannot upload the trial pair");
    }
  }
  const JobPtrs job{left, right, disp, vol, ws};
  const std::vector<Plan> cands = plan_candidates(p);
  constexpr int kWarm = 2, kReps = 5;
  float best_ms = 0.0f;
  for (size_t c = 0; c < cands.size(); ++c) {
    {
      std::lock_guard<std::mutex> lk(g_plan_mu);
      g_plans[plan_key(p)] = cands[c];
    }
    for (int r = 0; r < kWarm && rc == ZDT_OK; ++r) rc = solve_group(p, &job, 1, s);
    if (rc == ZDT_OK && hipEventRecord(e0, s) != hipSuccess) rc = fail(ZDT_EHIP, "zdt_autotune: event record");
    for (int r = 0; r < kReps && rc == ZDT_OK; ++r) rc = solve_group(p, &job, 1, s);
    float ms = 0.0f;
    if (rc == ZDT_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = fail(ZDT_EHIP, "zdt_autotune: timing failed");
    if (rc) break;
    if (c == 0 || ms < best_ms) {
      best_ms = ms;
      best = cands[c];
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (rc == ZDT_OK)
      g_plans[plan_key(p)] = best;
    else
      g_plans.erase(plan_key(p));
  }
  if (hipStreamSynchronize(s) != hipSuccess && rc == ZDT_OK) rc = fail(ZDT_EHIP, "zdt_autotune: stream sync");
  release();
  if (rc) return rc;
  if (chosen) *chosen = to_c(best);
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (!f) return fail(ZDT_EINVAL, "zdt_autotune: cannot append to %s", cache_path);
    std::fprintf(f, "zdt-plan %d %d %d %d %d : %d %d %d %d  (%.1f us)\n", p->width, p->height, p->max_disp,
                 p->radius, p->vol_dtype, best.h_lanes, best.h_seg, best.v_lanes, best.v_seg, 1000.0 * best_ms / kReps);
    std::fclose(f);
  }
  return ZDT_OK;
}

int zdt_i8_codec(const int16_t* values, uint8_t* codes, int16_t* decoded, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && (!values || !codes || !decoded)))
    return fail(ZDT_EINVAL, "zdt_i8_codec: bad arguments (n = %lld)", (long long)n);
  if (n == 0) return ZDT_OK;
  const int threads = 256;
  return launch("i8_codec", i8_codec_kernel, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0,
                (hipStream_t)stream, values, codes, decoded, n);
}

int zdt_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (on) {
    for (auto& r : g_prof_pending) {
      (void)hipEventDestroy(r.start);
      (void)hipEventDestroy(r.stop);
    }
    g_prof_pending.clear();
    g_prof_acc.clear();
  }
  g_prof_on = on != 0;
  return ZDT_OK;
}

int zdt_profile_collect(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof_pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
      return fail(ZDT_EHIP, "zdt_profile_collect: event query failed");
    ProfAcc* acc = nullptr;
    for (auto& e : g_prof_acc)
      if (e.first == r.name) acc = &e.second;
    if (!acc) {
      g_prof_acc.emplace_back(r.name, ProfAcc{});
      acc = &g_prof_acc.back().second;
    }
    acc->ms += ms;
    acc->n += 1;
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  g_prof_pending.clear();
  return (int)g_prof_acc.size();
}

int zdt_profile_entry(int index, const char** name, double* total_ms, int64_t* launches) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (index < 0 || index >= (int)g_prof_acc.size()) return fail(ZDT_EINVAL, "zdt_profile_entry: index out of range");
  if (name) *name = g_prof_acc[index].first.c_str();
  if (total_ms) *total_ms = g_prof_acc[index].second.ms;
  if (launches) *launches = g_prof_acc[index].second.n;
  return ZDT_OK;
}

}  // extern "C"
