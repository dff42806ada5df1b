// zdt_sgm.hip -- semi-global matching over a stored cost volume: the
// aggregation of the paper's system S1 (ZNCC costs scaled by T, then SGM with
// penalties P1 and P2; Sec. V-D, Table IV).  SGM itself the paper takes from
// its reference [r7]; this is its four-path form (left-right, right-left,
// top-bottom, bottom-top) with constant penalties:
//
//   L_r(p, d) = s C(p, d) + min( L_r(q, d), L_r(q, d -+ 1) + P1,
//                                min_k L_r(q, k) + P2 ) - min_k L_r(q, k)
//
// where q is the previous pixel on path r (L_r = s C on the first pixel) and
// the aggregated volume is S(p, d) = sum over the four paths.
//
//   sgm_line_kernel  one workgroup of two waves per line (a row for the
//                    horizontal paths, a column for the vertical ones); lanes
//                    map to disparities, DPL consecutive ones per lane.  Wave 0
//                    runs the path in increasing coordinate order, wave 1 in
//                    decreasing.  Each wave first covers its own half of the
//                    line, storing its path costs into the sum volume (rows)
//                    or adding them to what the row kernel stored (columns);
//                    after a workgroup barrier it continues into the half the
//                    other wave has just covered, adding its costs there.  The
//                    column kernel can take the WTA of the finished sums in the
//                    second half instead of storing them.
//
// Per pixel a wave needs L(d -+ 1) from the neighbouring lanes (DPP wave
// shifts) and min_k L (a DPP reduction); the recursion is serial along the
// line, so the cost (and stored-sum) loads run a ring of K pixels ahead.
#include "zdt_host.hpp"

namespace zdt {
namespace {

constexpr float kInf = __builtin_inff();

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dppf(float v, float id) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(id), __float_as_int(v), CTRL, ROWS, 0xF, false));
}

// Order-preserving map of floats onto int32 (its own inverse): minima can then
// run as integer DPP minimum steps with INT_MAX for lanes without a source.
__device__ __forceinline__ int fkey(float v) {
  const int b = __float_as_int(v);
  return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float funkey(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ int dpp_min(int v) {
  return min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, CTRL, ROWS, 0xF, false));
}

// Minimum key over the 64 lanes (wave-uniform result).
__device__ __forceinline__ int wave_min_key(int v) {
  v = dpp_min<0xB1>(v);        // quad_perm [1,0,3,2]
  v = dpp_min<0x4E>(v);        // quad_perm [2,3,0,1]
  v = dpp_min<0x141>(v);       // row_half_mirror
  v = dpp_min<0x140>(v);       // row_mirror
  v = dpp_min<0x142, 0xA>(v);  // row_bcast:15
  v = dpp_min<0x143, 0xC>(v);  // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}

// Disparities d = DPL * lane + k, k < DPL.  VEC: D is a multiple of DPL, so a
// lane's values are all valid or all padding and load as one vector (the
// volumes are 16-byte aligned, checked on the host).
template <int DPL, bool VEC>
struct Slot {
  float v[DPL];
};

// Loads a lane's DPL values of element type E (float, or _Float16 costs).
template <int DPL, bool VEC, typename E>
__device__ __forceinline__ void load_slot(Slot<DPL, VEC>& s, const E* base, int lane, int D) {
  if constexpr (VEC && DPL > 1) {
    typedef E V __attribute__((ext_vector_type(DPL)));
    const V x = *reinterpret_cast<const V*>(base + min(DPL * lane, D - DPL));
#pragma unroll
    for (int k = 0; k < DPL; ++k) s.v[k] = (float)x[k];
  } else {
#pragma unroll
    for (int k = 0; k < DPL; ++k) s.v[k] = (float)base[min(DPL * lane + k, D - 1)];
  }
}

template <int DPL, bool VEC, bool PAD>
__device__ __forceinline__ void store_slot(float* base, const float (&v)[DPL], int lane, int D) {
  if constexpr (VEC && DPL > 1) {
    using V = typename std::conditional<DPL == 2, float2, float4>::type;
    if (!PAD || DPL * lane < D) {
      V x;
      x.x = v[0];
      x.y = v[1];
      if constexpr (DPL == 4) {
        x.z = v[2];
        x.w = v[3];
      }
      *reinterpret_cast<V*>(base + DPL * lane) = x;
    }
  } else {
#pragma unroll
    for (int k = 0; k < DPL; ++k)
      if (!PAD || DPL * lane + k < D) base[DPL * lane + k] = v[k];
  }
}

// One pixel of a path: L <- s C + min(L, L(d -+ 1) + P1, m + P2) - m, then
// m <- min_d L.  pad[k] is -inf for a real disparity and +inf for padding, so
// that padding holds +inf and never wins a minimum (PAD: the wave has some).
// min(a, b) + P1 is formed as min(a + P1, b + P1), the same value under
// monotone rounding.
template <int DPL, bool PAD>
__device__ __forceinline__ void sgm_step(float (&L)[DPL], float& m, const float (&c)[DPL], const float (&pad)[DPL],
                                         float p1, float p2, float scale) {
  const float lo = dppf<0x138>(L[DPL - 1], kInf);  // wave_shr:1 -- L(d - 1) of this lane's first d
  const float hi = dppf<0x130>(L[0], kInf);        // wave_shl:1 -- L(d + 1) of its last d
  const float mp2 = m + p2;
  float up[DPL + 2];  // L(d) + P1 for d = first - 1 .. last + 1
  up[0] = lo + p1;
#pragma unroll
  for (int k = 0; k < DPL; ++k) up[k + 1] = L[k] + p1;
  up[DPL + 1] = hi + p1;
  float lm = kInf;
#pragma unroll
  for (int k = 0; k < DPL; ++k) {
    const float best = fminf(fminf(L[k], fminf(up[k], up[k + 2])), mp2);
    float v = fmaf(scale, c[k], best - m);
    if constexpr (PAD) v = fmaxf(v, pad[k]);
    L[k] = v;
    lm = fminf(lm, v);
  }
  m = funkey(wave_min_key(fkey(lm)));
}

// Smallest d holding the wave minimum of v (padding holds +inf).
template <int DPL>
__device__ __forceinline__ int wave_argmin(const float (&v)[DPL], int lane) {
  float lm = v[DPL - 1];
  int kk = DPL - 1;
#pragma unroll
  for (int k = DPL - 2; k >= 0; --k)
    if (v[k] <= lm) {
      lm = v[k];
      kk = k;
    }
  const int key = fkey(lm);
  const int gk = wave_min_key(key);
  const uint64_t hit = __ballot(key == gk);
  const int l0 = __builtin_ctzll(hit);  // hit != 0: the lane the minimum came from
  return DPL * l0 + __builtin_amdgcn_readlane(kk, l0);
}

// Pixel ring depth: K pixels of cost (and of stored sums) in flight per wave.
// With 16-bit costs a pixel's loads are fewer bytes, and the row pass (one
// wave per path of a row, fewer waves than SIMDs) is bound by the loads in
// flight: twice the depth took its time from 246 to 226 us at 1280x384,
// D = 128, while the FP32-cost passes, already at the memory's rate, gained
// nothing from it.
template <int DPL, typename E>
constexpr int ring_depth() {
  constexpr int k = DPL == 1 ? 16 : (DPL == 2 ? 12 : 8);
  return sizeof(E) == 2 ? 2 * k : k;
}

// Run `count` pixels of one path, starting at pixel p0 and stepping by dp.
// LOADS: add the sum stored at each pixel.  Then either store the result
// (STORES) or write the WTA of it (WTA).
template <typename E, int DPL, bool VEC, bool PAD, bool LOADS, bool STORES, bool WTA>
__device__ __forceinline__ void sgm_run(const SgmArgs& a, int p0, int dp, int count, float (&L)[DPL], float& m,
                                        const float (&pad)[DPL], int lane) {
  constexpr int K = ring_depth<DPL, E>();
  if (count <= 0) return;
  const int D = a.D;
  const E* cost = static_cast<const E*>(a.cost);
  const int last = count - 1;
  Slot<DPL, VEC> cb[K], sb[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int pix = p0 + min(j, last) * dp;
    load_slot(cb[j], cost + (size_t)pix * D, lane, D);
    if constexpr (LOADS) load_slot(sb[j], a.sum + (size_t)pix * D, lane, D);
  }
  auto body = [&](int i, Slot<DPL, VEC>& c, Slot<DPL, VEC>& s) {
    sgm_step<DPL, PAD>(L, m, c.v, pad, a.p1, a.p2, a.scale);
    const int pix = p0 + i * dp;
    float out[DPL];
#pragma unroll
    for (int k = 0; k < DPL; ++k) out[k] = LOADS ? s.v[k] + L[k] : L[k];
    if constexpr (STORES) store_slot<DPL, VEC, PAD>(a.sum + (size_t)pix * D, out, lane, D);
    if constexpr (WTA) {
      const int d = wave_argmin<DPL>(out, lane);
      if (lane == 0) a.disp[pix] = d;
    }
  };
  int i0 = 0;
  for (; i0 + K <= count; i0 += K) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      body(i0 + j, cb[j], sb[j]);
      const int pix = p0 + min(i0 + j + K, last) * dp;
      load_slot(cb[j], cost + (size_t)pix * D, lane, D);
      if constexpr (LOADS) load_slot(sb[j], a.sum + (size_t)pix * D, lane, D);
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (i0 + j < count) body(i0 + j, cb[j], sb[j]);
}

template <typename E, int DPL, bool VEC, bool PAD, bool VERT, bool WTA>
__global__ __launch_bounds__(128) void sgm_line_kernel(SgmArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const bool fwd = threadIdx.x < kWave;
  const int line = blockIdx.x;
  const int n = VERT ? a.H : a.W;
  const int stride = VERT ? a.W : 1;
  const int base = VERT ? line : line * a.W;  // pixel index of the line's first pixel
  const int half = n / 2;                     // wave 0 starts on [0, half), wave 1 on [half, n)
  float pad[DPL], L[DPL];
#pragma unroll
  for (int k = 0; k < DPL; ++k) {
    const bool ok = !PAD || DPL * lane + k < a.D;
    pad[k] = ok ? -kInf : kInf;
    L[k] = ok ? 0.0f : kInf;  // with m = 0 the first step gives L = s C
  }
  float m = 0.0f;
  if (fwd)
    sgm_run<E, DPL, VEC, PAD, VERT, true, false>(a, base, stride, half, L, m, pad, lane);
  else
    sgm_run<E, DPL, VEC, PAD, VERT, true, false>(a, base + (n - 1) * stride, -stride, n - half, L, m, pad, lane);
  __syncthreads();  // each half now holds the other wave's contribution
  if (fwd)
    sgm_run<E, DPL, VEC, PAD, true, !WTA, WTA>(a, base + half * stride, stride, n - half, L, m, pad, lane);
  else
    sgm_run<E, DPL, VEC, PAD, true, !WTA, WTA>(a, base + (half - 1) * stride, -stride, half, L, m, pad, lane);
}

template <typename E, int DPL, bool VEC, bool PAD>
int run_sgm(const SgmArgs& a, bool vert, bool wta, hipStream_t s) {
  const dim3 block(2 * kWave);
  if (!vert) return launch("sgm_rows", sgm_line_kernel<E, DPL, VEC, PAD, false, false>, dim3(a.H), block, 0, s, a);
  if (!wta) return launch("sgm_cols", sgm_line_kernel<E, DPL, VEC, PAD, true, false>, dim3(a.W), block, 0, s, a);
  return launch("sgm_cols_wta", sgm_line_kernel<E, DPL, VEC, PAD, true, true>, dim3(a.W), block, 0, s, a);
}

template <typename E>
int dispatch_sgm_t(const SgmArgs& a, bool vert, bool wta, hipStream_t s) {
  const int dpl = (a.D + kWave - 1) / kWave;
  const bool vec = a.D % dpl == 0, pad = a.D < dpl * kWave;
  switch (dpl) {
    case 1: return pad ? run_sgm<E, 1, true, true>(a, vert, wta, s) : run_sgm<E, 1, true, false>(a, vert, wta, s);
    case 2:
      if (!pad) return run_sgm<E, 2, true, false>(a, vert, wta, s);
      return vec ? run_sgm<E, 2, true, true>(a, vert, wta, s) : run_sgm<E, 2, false, true>(a, vert, wta, s);
    case 3: return pad ? run_sgm<E, 3, false, true>(a, vert, wta, s) : run_sgm<E, 3, false, false>(a, vert, wta, s);
    case 4:
      if (!pad) return run_sgm<E, 4, true, false>(a, vert, wta, s);
      return vec ? run_sgm<E, 4, true, true>(a, vert, wta, s) : run_sgm<E, 4, false, true>(a, vert, wta, s);
  }
  return fail(ZDT_EUNSUPPORTED, "sgm: max_disp %d > %d", a.D, 4 * kWave);
}

}  // namespace

int dispatch_sgm(const SgmArgs& a, bool vert, bool wta, hipStream_t s) {
  return a.cost_f16 ? dispatch_sgm_t<_Float16>(a, vert, wta, s) : dispatch_sgm_t<float>(a, vert, wta, s);
}

}  // namespace zdt
