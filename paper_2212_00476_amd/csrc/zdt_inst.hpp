// zdt_inst.hpp -- kernel instances and dispatch for one volume element type.
// Included once by each zdt_inst_<type>.hip with ZDT_ELEM and ZDT_SUFFIX set.
#pragma once
#include <type_traits>

#include "zdt_host.hpp"

namespace zdt {
namespace inst {

template <int R, int SEG, int LPS, typename T, int MODE>
int run_h(const HArgs& a, const HJobs& jobs, int n, hipStream_t s) {
  constexpr bool kDT = MODE == kCostHPair || MODE == kHPair;
  const int wl = kDT ? (kWave / LPS) * kMaxWaves * SEG : a.W;  // as in hpass_kernel
  const HLayout lay = h_layout(wl, R, LPS, SEG, MODE != kHPair, kDT, std::is_same<T, f16x>::value || is_int_vol<T>());
  static const char* const names[] = {"zncc_sums", "zncc_cost", "zncc_hpair", "dt_hpair"};
  const int spw = kWave / LPS;
  const int nw = (a.nseg + spw - 1) / spw;
  HArgs b = a;
  // the Int8 reference launch covers disparity chunk 0 only
  b.nchunks = a.ref_role == kRefL2ROut ? 1 : (a.D + LPS - 1) / LPS;
  dim3 grid(b.nchunks, a.H, n);
  if constexpr (kDT)  // tile order of the H pass (h_order)
    grid = dim3((unsigned)(h_order<sizeof(T)>() == 1 ? pair_grid(a.H, b.nchunks) : xcd_grid(a.H * b.nchunks)), 1, n);
  return launch(names[MODE], hpass_kernel<R, SEG, LPS, T, MODE>, grid, dim3(kWave * nw), (size_t)lay.words * 4, s, b,
                jobs);
}

template <int R, int LPS, typename T, int MODE>
int run_h_seg(int seg, const HArgs& a, const HJobs& jobs, int n, hipStream_t s) {
  if constexpr (LPS == 32) {
    switch (seg) {
      case 8: return run_h<R, 8, LPS, T, MODE>(a, jobs, n, s);
      case 20: return run_h<R, 20, LPS, T, MODE>(a, jobs, n, s);
      case 40: return run_h<R, 40, LPS, T, MODE>(a, jobs, n, s);
      case 60: return run_h<R, 60, LPS, T, MODE>(a, jobs, n, s);
    }
  } else {
    switch (seg) {
      case 16: return run_h<R, 16, LPS, T, MODE>(a, jobs, n, s);
      case 40: return run_h<R, 40, LPS, T, MODE>(a, jobs, n, s);
      case 80: return run_h<R, 80, LPS, T, MODE>(a, jobs, n, s);
    }
  }
  return fail(ZDT_EUNSUPPORTED, "no H-pass instance for segment length %d", seg);
}

// Streaming modes (sums, raw cost) keep no per-segment registers: SEG = 0.
template <typename T, int MODE, int LPS>
int run_h_radius(int R, int seg, const HArgs& a, const HJobs& jobs, int n, hipStream_t s) {
  constexpr bool stream = MODE == kSums || MODE == kCost;
  switch (R) {
#define ZDT_CASE(RR)                                                \
  case RR:                                                          \
    if constexpr (stream) return run_h<RR, 0, 64, T, MODE>(a, jobs, n, s); \
    else return run_h_seg<RR, LPS, T, MODE>(seg, a, jobs, n, s);
    ZDT_CASE(0) ZDT_CASE(1) ZDT_CASE(2) ZDT_CASE(3) ZDT_CASE(4) ZDT_CASE(5) ZDT_CASE(6) ZDT_CASE(7)
#undef ZDT_CASE
  }
  return fail(ZDT_EUNSUPPORTED, "no H-pass instance for radius %d", R);
}

template <int SEG, bool FULL, typename T, int LPS, bool WTA>
int run_v(const VArgs& a, const VJobs& jobs, int n, hipStream_t s) {
  VArgs b = a;
  b.nchunks = (a.D + LPS - 1) / LPS;
  const dim3 grid((unsigned)xcd_grid(a.W * b.nchunks), 1, n);  // (column, chunk) tiles in xcd_tile order
  const int nw = a.nseg / (kWave / LPS);
  return launch(WTA ? "dt_vpair_wta" : "dt_vpair", vpass_kernel<SEG, FULL, T, LPS, WTA>, grid, dim3(kWave * nw),
                (size_t)v_lds_words(a.H, SEG, std::is_same<T, f16x>::value, is_int_vol<T>()) * 4, s, b, jobs);
}

template <typename T, bool WTA>
int run_v_seg(int seg, int lps, bool full, const VArgs& a, const VJobs& jobs, int n, hipStream_t s) {
  if (lps == 32) {
    if (!full) return fail(ZDT_EUNSUPPORTED, "V pass: 32-lane segments must be full");
    switch (seg) {
#define ZDT_CASE(SS) \
  case SS: return run_v<SS, true, T, 32, WTA>(a, jobs, n, s);
      ZDT_CASE(12) ZDT_CASE(24) ZDT_CASE(36)
#undef ZDT_CASE
    }
  } else {
    switch (seg) {
#define ZDT_CASE(SS)                                                  \
  case SS:                                                            \
    return full ? run_v<SS, true, T, 64, WTA>(a, jobs, n, s)          \
                : run_v<SS, false, T, 64, WTA>(a, jobs, n, s);
      ZDT_CASE(8) ZDT_CASE(12) ZDT_CASE(24) ZDT_CASE(48) ZDT_CASE(72)
#undef ZDT_CASE
    }
  }
  return fail(ZDT_EUNSUPPORTED, "no V-pass instance for segment length %d, %d lanes", seg, lps);
}

}  // namespace inst
}  // namespace zdt

#define ZDT_CAT2(a, b) a##b
#define ZDT_CAT(a, b) ZDT_CAT2(a, b)

namespace zdt {

int ZDT_CAT(dispatch_h_, ZDT_SUFFIX)(int mode, int R, int seg, int lps, const HArgs& a, const HJobs& jobs, int n,
                                     hipStream_t s) {
  using T = ZDT_ELEM;
  constexpr bool f32 = std::is_same<T, float>::value;
  constexpr bool f16x_ = std::is_same<T, f16x>::value;
  switch (mode) {
    case kCost:
      if constexpr (!f16x_ && !std::is_same<T, i8c>::value)
        return inst::run_h_radius<T, kCost, 64>(R, seg, a, jobs, n, s);
      break;
    case kCostHPair:
      if (lps == 32) return inst::run_h_radius<T, kCostHPair, 32>(R, seg, a, jobs, n, s);
      if (lps == 64) return inst::run_h_radius<T, kCostHPair, 64>(R, seg, a, jobs, n, s);
      break;
    case kHPair:
      if (lps == 32) return inst::run_h_seg<0, 32, T, kHPair>(seg, a, jobs, n, s);
      if (lps == 64) return inst::run_h_seg<0, 64, T, kHPair>(seg, a, jobs, n, s);
      break;
    case kSums:
      if constexpr (f32) return inst::run_h_radius<T, kSums, 64>(R, seg, a, jobs, n, s);
      break;
  }
  return fail(ZDT_EUNSUPPORTED, "no H-pass instance for mode %d, %d lanes per segment", mode, lps);
}

int ZDT_CAT(dispatch_v_, ZDT_SUFFIX)(int seg, int lps, bool wta, const VArgs& a, const VJobs& jobs, int n,
                                     hipStream_t s) {
  using T = ZDT_ELEM;
  const bool full = a.segl == seg && a.nseg * seg == a.H;
  if (!wta) return inst::run_v_seg<T, false>(seg, lps, full, a, jobs, n, s);
  return inst::run_v_seg<T, true>(seg, lps, full, a, jobs, n, s);
}

int ZDT_CAT(dispatch_wta_, ZDT_SUFFIX)(const void* vol, int npix, int D, int32_t* disp, hipStream_t s) {
  using T = ZDT_ELEM;
  if constexpr (std::is_same<T, f16x>::value) {
    return fail(ZDT_EUNSUPPORTED, "no standalone WTA over an exponent-scaled volume");
  } else {
  const int threads = 256, waves_per_block = threads / kWave;
  int blocks = (npix + waves_per_block - 1) / waves_per_block;
  if (blocks > 8192) blocks = 8192;
  return launch("wta", wta_kernel<T>, dim3(blocks), dim3(threads), 0, s, (const T*)vol, npix, D, disp);
  }
}

}  // namespace zdt
