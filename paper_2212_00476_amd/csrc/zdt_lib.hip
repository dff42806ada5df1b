// zdt_lib.hip -- the C ABI declared in include/zdt.h.
//
// Validation, launch-shape selection and per-launch HIP-event timing.  The
// device work is in zdt_device.hpp; its compiled instances live in
// zdt_inst_<type>.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
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
std::unordered_map<const void*, int> g_kernel_ok;  // kernel -> ZDT_OK or a ZDT_E* code
}  // namespace

int check_kernel(const void* kernel, const char* name) {
  std::lock_guard<std::mutex> lk(g_kernel_mu);
  auto it = g_kernel_ok.find(kernel);
  if (it != g_kernel_ok.end()) {
    if (it->second != ZDT_OK) fail(it->second, "%s: kernel was refused (per-lane scratch too large)", name);
    return it->second;
  }
  hipFuncAttributes attr{};
  const hipError_t e = hipFuncGetAttributes(&attr, kernel);
  if (e != hipSuccess) return fail(ZDT_EHIP, "%s: hipFuncGetAttributes: %s", name, hipGetErrorString(e));
  int rc = ZDT_OK;
  if (attr.localSizeBytes > kMaxScratchBytes)
    rc = fail(ZDT_EUNSUPPORTED, "%s: kernel needs %zu B of scratch per lane (limit %d)", name,
              (size_t)attr.localSizeBytes, kMaxScratchBytes);
  g_kernel_ok.emplace(kernel, rc);
  return rc;
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

bool prof_begin(ProfRec& rec, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return false;
  }
  if (hipEventCreate(&rec.start) != hipSuccess || hipEventCreate(&rec.stop) != hipSuccess ||
      hipEventRecord(rec.start, s) != hipSuccess)
    return false;
  return true;
}

void prof_end(ProfRec& rec, hipStream_t s) {
  if (hipEventRecord(rec.stop, s) != hipSuccess) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_pending.push_back(rec);
}

}  // namespace zdt

using namespace zdt;

namespace {

constexpr int kMaxRadius = 6;

size_t dtype_size(int t) { return t == ZDT_F32 ? 4 : 2; }

int check_params(const zdt_params* p, const char* who) {
  if (!p) return fail(ZDT_EINVAL, "%s: params is NULL", who);
  if (p->width < 1 || p->height < 1) return fail(ZDT_EINVAL, "%s: width/height must be >= 1", who);
  if (p->pitch < p->width) return fail(ZDT_EINVAL, "%s: pitch %d < width %d", who, p->pitch, p->width);
  if (p->max_disp < 1) return fail(ZDT_EINVAL, "%s: max_disp must be >= 1", who);
  if (p->radius < 0) return fail(ZDT_EINVAL, "%s: radius must be >= 0", who);
  if (p->radius > kMaxRadius)
    return fail(ZDT_EUNSUPPORTED, "%s: radius %d > %d (int32 sums need l <= 13)", who, p->radius, kMaxRadius);
  if (!(p->sigma_s > 0.0f) || std::isinf(p->sigma_s))
    return fail(ZDT_EINVAL, "%s: sigma_s must be finite and > 0", who);
  if (!(p->sigma_r > 0.0f)) return fail(ZDT_EINVAL, "%s: sigma_r must be > 0 (or +inf)", who);
  if (p->dt_iters < 0) return fail(ZDT_EINVAL, "%s: dt_iters must be >= 0", who);
  if (p->vol_dtype < ZDT_F32 || p->vol_dtype > ZDT_BF16)
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

// A line of n values split into nseg <= maxseg segments of segl <= seg values
// (the smallest compiled seg that fits).
struct Split {
  int seg, segl, nseg;
};

Split split_line(int n, const int* segs, int nsegs, int maxseg) {
  for (int i = 0; i < nsegs; ++i)
    if (n <= maxseg * segs[i]) {
      const int n0 = (n + segs[i] - 1) / segs[i];
      const int segl = (n + n0 - 1) / n0;
      return {segs[i], segl, (n + segl - 1) / segl};
    }
  return {0, 0, 0};
}

Split h_split(const zdt_params* p, int lps, int mode) {
  if (mode == kSums || mode == kCost) {  // streamed: any segment length, 16 waves
    const int segl = (p->width + kMaxWaves - 1) / kMaxWaves;
    return {0, segl, (p->width + segl - 1) / segl};
  }
  if (lps == 32) {
    const int seg = h_full_seg32(p->width);
    return {seg, seg, p->width / seg};
  }
  return split_line(p->width, kHSegs64, kNumHSegs64, kMaxWaves);
}
Split v_split(const zdt_params* p) { return split_line(p->height, kVSegs, kNumVSegs, kMaxWaves); }

bool normalized(const zdt_params* p) { return (p->flags & ZDT_FLAG_NORMALIZE) || p->vol_dtype != ZDT_F32; }

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

HArgs make_hargs(const zdt_params* p, const uint8_t* left, const uint8_t* right, const uint8_t* guide, void* vol,
                 float out_scale, const Split& sp) {
  HArgs a{};
  a.left = left;
  a.right = right;
  a.guide = guide;
  a.pitch = p->pitch;
  a.W = p->width;
  a.H = p->height;
  a.D = p->max_disp;
  a.inv_sigma_s = 1.0f / p->sigma_s;
  a.range_coef = range_coef(p);
  a.out_scale = out_scale;
  a.vol = vol;
  a.segl = sp.segl;
  a.nseg = sp.nseg;
  return a;
}

VArgs make_vargs(const zdt_params* p, const uint8_t* guide, void* vol, float out_scale, const Split& sp) {
  VArgs a{};
  a.guide = guide;
  a.pitch = p->pitch;
  a.W = p->width;
  a.H = p->height;
  a.D = p->max_disp;
  a.inv_sigma_s = 1.0f / p->sigma_s;
  a.range_coef = range_coef(p);
  a.out_scale = out_scale;
  a.vol = vol;
  a.segl = sp.segl;
  a.nw = sp.nseg;
  return a;
}

// Launch an H-pass mode: the lane layout follows the volume type and mode.
int run_h_mode(const zdt_params* p, int dtype, int mode, const uint8_t* left, const uint8_t* right,
               const uint8_t* guide, void* vol, float scale, int8_t* ex, hipStream_t s, HArgs* extra = nullptr) {
  const int lps = h_lps(dtype, mode, p->width);
  const Split sp = h_split(p, lps, mode);
  HArgs a = make_hargs(p, left, right, guide, vol, scale, sp);
  a.ex = ex;
  if (extra) {
    a.s_rt = extra->s_rt;
    a.s_l = extra->s_l;
    a.s_ll = extra->s_ll;
    a.s_t = extra->s_t;
    a.s_tt = extra->s_tt;
  }
  const int R = mode == kHPair ? 0 : p->radius;
  switch (dtype) {
    case ZDT_F32: return dispatch_h_f32(mode, R, sp.seg, lps, a, s);
    case ZDT_F16:
      return ex ? dispatch_h_f16x(mode, R, sp.seg, lps, a, s) : dispatch_h_f16(mode, R, sp.seg, lps, a, s);
    case ZDT_BF16: return dispatch_h_bf16(mode, R, sp.seg, lps, a, s);
  }
  return fail(ZDT_EINVAL, "bad dtype %d", dtype);
}

int dispatch_v(int dtype, int seg, int dpl, bool wta, const VArgs& a, int nchunks, hipStream_t s) {
  switch (dtype) {
    case ZDT_F32: return dispatch_v_f32(seg, dpl, wta, a, nchunks, s);
    case ZDT_F16:
      return a.ex ? dispatch_v_f16x(seg, dpl, wta, a, nchunks, s) : dispatch_v_f16(seg, dpl, wta, a, nchunks, s);
    case ZDT_BF16: return dispatch_v_bf16(seg, dpl, wta, a, nchunks, s);
  }
  return fail(ZDT_EINVAL, "bad dtype %d", dtype);
}

int dispatch_wta(int dtype, const void* vol, int npix, int D, int32_t* disp, hipStream_t s) {
  switch (dtype) {
    case ZDT_F32: return dispatch_wta_f32(vol, npix, D, disp, s);
    case ZDT_F16: return dispatch_wta_f16(vol, npix, D, disp, s);
    case ZDT_BF16: return dispatch_wta_bf16(vol, npix, D, disp, s);
  }
  return fail(ZDT_EINVAL, "bad dtype %d", dtype);
}

// Shape of the WTA-fused V pass: DPL disparities per lane and the number of
// disparity chunks (several chunks need the partial-minimum workspace).
struct VWta {
  int dpl, nchunks;
};
VWta v_wta_shape(const zdt_params* p, int seg) {
  (void)seg;
  // one disparity per lane keeps the kernel at two workgroups per CU; several
  // 64-disparity chunks are combined by a small second kernel
  return {1, (p->max_disp + kWave - 1) / kWave};
}

// Workspace of stereo_solve: the FP16 exponent map, then the WTA partial minima.
struct WsLayout {
  size_t ex, part_val, part_idx, total;
};
size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }
WsLayout ws_layout(const zdt_params* p) {
  WsLayout L{};
  const size_t npix = (size_t)p->width * p->height;
  const size_t nck = (size_t)(p->max_disp + kExpChunk - 1) / kExpChunk;
  size_t o = 0;
  if (p->vol_dtype == ZDT_F16 && p->dt_iters > 0) {
    L.ex = o;
    o += align256(npix * nck);
  }
  const VWta vw = v_wta_shape(p, v_split(p).seg);
  if (p->dt_iters > 0 && vw.nchunks > 1) {
    L.part_val = o;
    o += align256((size_t)vw.nchunks * npix * sizeof(float));
    L.part_idx = o;
    o += align256((size_t)vw.nchunks * npix * sizeof(int32_t));
  }
  L.total = o;
  return L;
}

int run_hpair(const zdt_params* p, const uint8_t* guide, void* vol, float scale, int8_t* ex, hipStream_t s) {
  return run_h_mode(p, p->vol_dtype, kHPair, nullptr, nullptr, guide, vol, scale, ex, s);
}

int run_vpair(const zdt_params* p, const uint8_t* guide, void* vol, float scale, int8_t* ex, hipStream_t s) {
  const Split sp = v_split(p);
  VArgs a = make_vargs(p, guide, vol, scale, sp);
  a.ex = ex;
  return dispatch_v(p->vol_dtype, sp.seg, 1, false, a, (p->max_disp + kWave - 1) / kWave, s);
}

int run_vpair_wta(const zdt_params* p, const uint8_t* guide, void* vol, float scale, int8_t* ex, int32_t* disp,
                  void* ws, hipStream_t s) {
  const Split sp = v_split(p);
  const VWta vw = v_wta_shape(p, sp.seg);
  VArgs va = make_vargs(p, guide, vol, scale, sp);
  va.ex = ex;
  if (vw.nchunks == 1) {
    va.disp = disp;
    return dispatch_v(p->vol_dtype, sp.seg, vw.dpl, true, va, 1, s);
  }
  const WsLayout L = ws_layout(p);
  const size_t npix = (size_t)p->width * p->height;
  va.part_val = (float*)((char*)ws + L.part_val);
  va.part_idx = (int32_t*)((char*)ws + L.part_idx);
  int rc = dispatch_v(p->vol_dtype, sp.seg, vw.dpl, true, va, vw.nchunks, s);
  if (rc) return rc;
  const int threads = 256;
  return launch("wta_combine", wta_combine_kernel, dim3((unsigned)((npix + threads - 1) / threads)), dim3(threads), 0,
                s, (const float*)va.part_val, (const int32_t*)va.part_idx, vw.nchunks, (int)npix, disp);
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
  return run_h_mode(p, p->vol_dtype, kCost, left, right, nullptr, cost, 1.0f, nullptr, (hipStream_t)stream);
}

int zncc_window_sums(const zdt_params* p, const uint8_t* left, const uint8_t* right, int32_t* s_l, int32_t* s_ll,
                     int32_t* s_t, int32_t* s_tt, int32_t* s_rt, void* stream) {
  int rc = check_params(p, "zncc_window_sums");
  if (rc) return rc;
  if (!left || !right) return fail(ZDT_EINVAL, "zncc_window_sums: NULL image pointer");
  HArgs sums{};
  sums.s_rt = s_rt;
  sums.s_l = s_l;
  sums.s_ll = s_ll;
  sums.s_t = s_t;
  sums.s_tt = s_tt;
  return run_h_mode(p, ZDT_F32, kSums, left, right, nullptr, nullptr, 1.0f, nullptr, (hipStream_t)stream, &sums);
}

int dt_aggregate(const zdt_params* p, const uint8_t* guide, void* cost, double* applied_scale, void* stream) {
  int rc = check_params(p, "dt_aggregate");
  if (rc) return rc;
  if (!guide || !cost) return fail(ZDT_EINVAL, "dt_aggregate: NULL guide or volume pointer");
  hipStream_t s = (hipStream_t)stream;
  const float sc = pair_scale(p);
  for (int it = 0; it < p->dt_iters; ++it) {
    if ((rc = run_hpair(p, guide, cost, sc, nullptr, s))) return rc;
    if ((rc = run_vpair(p, guide, cost, sc, nullptr, s))) return rc;
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
  int rc = check_params(p, "stereo_solve");
  if (rc) return rc;
  if (!left || !right || !disp || !vol)
    return fail(ZDT_EINVAL, "stereo_solve: NULL image, disparity or volume pointer");
  hipStream_t s = (hipStream_t)stream;
  const uint8_t* guide = (p->flags & ZDT_FLAG_GUIDE_TARGET) ? right : left;
  if (p->dt_iters == 0) {
    if ((rc = run_h_mode(p, p->vol_dtype, kCost, left, right, nullptr, vol, 1.0f, nullptr, s))) return rc;
    return dispatch_wta(p->vol_dtype, vol, p->width * p->height, p->max_disp, disp, s);
  }
  const WsLayout L = ws_layout(p);
  if (L.total && !ws) return fail(ZDT_EINVAL, "stereo_solve: a workspace of %zu B is required", L.total);
  // An FP16 working volume keeps per-(pixel, chunk) exponents and needs no
  // global scale; the other types take the (1-K)-per-pass normalisation.
  int8_t* ex = p->vol_dtype == ZDT_F16 ? (int8_t*)((char*)ws + L.ex) : nullptr;
  const float sc = ex ? 1.0f : pair_scale(p);
  // sweep 1: cost fused with L, R; then U, D.  Sweeps 2..I: L, R; U, D.  The
  // last U, D pair carries the WTA and writes no volume.
  if ((rc = run_h_mode(p, p->vol_dtype, kCostHPair, left, right, guide, vol, sc, ex, s))) return rc;
  for (int it = 0; it < p->dt_iters; ++it) {
    if (it > 0 && (rc = run_hpair(p, guide, vol, sc, ex, s))) return rc;
    if (it + 1 < p->dt_iters) {
      if ((rc = run_vpair(p, guide, vol, sc, ex, s))) return rc;
    } else if ((rc = run_vpair_wta(p, guide, vol, sc, ex, disp, ws, s))) {
      return rc;
    }
  }
  return ZDT_OK;
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
