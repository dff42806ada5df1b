// zdt_host.hpp -- host-side helpers shared by the C-ABI translation unit and
// the per-dtype kernel-instance translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "zdt.h"
#include "zdt_device.hpp"

namespace zdt {

// Record an error message for zdt_last_error() and return `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// Per-launch event timing (active between zdt_profile_enable(1) and (0)).
struct ProfRec {
  const char* name;
  hipEvent_t start, stop;
};
bool prof_begin(ProfRec& rec, hipStream_t s);
void prof_end(ProfRec& rec, hipStream_t s);

// Every kernel keeps its working set in registers and LDS; one that needs
// more per-lane scratch than this is refused with ZDT_EUNSUPPORTED rather than
// launched.  The check, and raising a kernel's dynamic-LDS limit above 64 KB,
// happen on the first launch that needs them only, so a warmed-up sequence of
// launches can be captured into a graph with nothing else in between.
constexpr int kMaxScratchBytes = 1024;
int prepare_kernel(const void* kernel, const char* name, size_t lds);

template <typename Kernel, typename... A>
int launch(const char* name, Kernel kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, A... args) {
  if (const int rc = prepare_kernel((const void*)kernel, name, lds)) return rc;
  ProfRec rec{name, nullptr, nullptr};
  const bool prof = prof_begin(rec, s);
  hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
  hipError_t e = hipGetLastError();
  if (prof) prof_end(rec, s);
  if (e != hipSuccess) return fail(ZDT_EHIP, "%s: launch failed: %s", name, hipGetErrorString(e));
  return ZDT_OK;
}

// Segment lengths (values per lane) compiled for the H and V passes.  A pass
// gives each wave two segments of 32 disparities when the line splits into
// full segments (a 128-byte line per half-wave for FP32, half a line for
// 16-bit volumes, whose two chunks then share an XCD), else one of 64.
constexpr int kHSegs32[] = {8, 20, 40, 60};  // LPS = 32: up to 32 segments per row
constexpr int kHSegs64[] = {16, 40, 80};      // LPS = 64: up to 16 segments per row
constexpr int kVSegs[] = {8, 12, 24, 48, 72};  // 64 lanes: up to 16 segments per column
constexpr int kVSegs32[] = {12, 24, 36};         // 32 lanes: up to 32 full segments per column
constexpr int kNumHSegs64 = 3, kNumVSegs = 5, kNumVSegs32 = 3;
// FP32 H pairs take two segments per wave when the row splits into an even
// number (<= 32) of full segments of a compiled length; otherwise one.
inline bool h_seg32_fits(int W, int seg) { return W % seg == 0 && (W / seg) % 2 == 0 && W / seg <= 2 * kMaxWaves; }
inline int h_full_seg32(int W) {
  for (int seg : kHSegs32)
    if (h_seg32_fits(W, seg)) return seg;
  return 0;
}
// The default among them: the longest of up to 40 values that still leaves at
// least 12 segments (fewer carries to compose; measured 1-8 % faster than
// 20-value segments at widths 480 and 640), else the shortest that fits
// (narrower rows need the waves: 40-value segments at width 320 were 6-11 %
// slower).
inline int h_default_seg32(int W) {
  int best = 0;
  for (int seg : kHSegs32)
    if (seg <= 40 && h_seg32_fits(W, seg) && W / seg >= 12) best = seg;
  return best ? best : h_full_seg32(W);
}

// Kernel dispatch, one set per volume element type (defined in zdt_inst_*.hip).
#define ZDT_DECLARE_DISPATCH(SUFFIX)                                                                           \
  int dispatch_h_##SUFFIX(int mode, int R, int seg, int lps, const HArgs& a, const HJobs& jobs, int n,        \
                          hipStream_t s);                                                                     \
  int dispatch_v_##SUFFIX(int seg, int lps, bool wta, const VArgs& a, const VJobs& jobs, int n, hipStream_t s); \
  int dispatch_wta_##SUFFIX(const void* vol, int npix, int D, int32_t* disp, hipStream_t s);
ZDT_DECLARE_DISPATCH(f32)
ZDT_DECLARE_DISPATCH(f16)
ZDT_DECLARE_DISPATCH(bf16)
ZDT_DECLARE_DISPATCH(f16x)
ZDT_DECLARE_DISPATCH(i16)
ZDT_DECLARE_DISPATCH(i8)
#undef ZDT_DECLARE_DISPATCH

// Semi-global matching over a cost volume [H][W][D], FP32 or (cost_f16) FP16
// (zdt_sgm.hip).  The FP32 `sum` receives the row paths (vert = false), then
// the column paths are added in place (vert = true), or with wta their sums go
// straight into `disp`.
struct SgmArgs {
  const void* cost;
  int cost_f16;
  float* sum;
  int32_t* disp;
  int W, H, D;
  float p1, p2, scale;
};
int dispatch_sgm(const SgmArgs& a, bool vert, bool wta, hipStream_t s);

// Window sums by integral images (zdt_integral.hip): 32-bit words of one
// integral array of image 0 (reference) or 1 (target), and the whole pass.
size_t integral_words(int W, int H, int D, int r, int image);
int integral_window_sums(const uint8_t* left, const uint8_t* right, int pitch, int W, int H, int D, int r,
                         int32_t* s_l, int32_t* s_ll, int32_t* s_t, int32_t* s_tt, void* ws, hipStream_t s);

}  // namespace zdt
