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

// Minimum over the 64 lanes (lanes without a source contribute +inf).
__device__ __forceinline__ float wave_minf(float v) {
  v = fminf(v, dppf<0xB1>(v, kInf));         // quad_perm [1,0,3,2]
  v = fminf(v, dppf<0x4E>(v, kInf));         // quad_perm [2,3,0,1]
  v = fminf(v, dppf<0x141>(v, kInf));        // row_half_mirror
  v = fminf(v, dppf<0x140>(v, kInf));        // row_mirror
  v = fminf(v, dppf<0x142, 0xA>(v, kInf));   // row_bcast:15
  v = fminf(v, dppf<0x143, 0xC>(v, kInf));   // row_bcast:31
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Disparities d = DPL * lane + k, k < DPL.  VEC: D is a multiple of DPL, so a
// lane's values are all valid or all padding and load as one vector.
template <int DPL, bool VEC>
struct Slot {
  float v[DPL];
};

template <int DPL, bool VEC>
__device__ __forceinline__ void load_slot(Slot<DPL, VEC>& s, const float* base, int lane, int D) {
  if constexpr (VEC && DPL > 1) {
    using V = typename std::conditional<DPL == 2, float2, float4>::type;
    const int o = min(DPL * lane, D - DPL);
    const V x = *reinterpret_cast<const V*>(base + o);
    s.v[0] = x.x;
    s.v[1] = x.y;
    if constexpr (DPL == 4) {
      s.v[2] = x.z;
      s.v[3] = x.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < DPL; ++k) s.v[k] = base[min(DPL * lane + k, D - 1)];
  }
}

template <int DPL, bool VEC>
__device__ __forceinline__ void store_slot(float* base, const float (&v)[DPL], int lane, int D) {
  if constexpr (VEC && DPL > 1) {
    using V = typename std::conditional<DPL == 2, float2, float4>::type;
    if (DPL * lane < D) {
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
      if (DPL * lane + k < D) base[DPL * lane + k] = v[k];
  }
}

// One pixel of a path: L <- s C + min(L, L(d -+ 1) + P1, m + P2) - m, then
// m <- min_d L.  Padding disparities hold +inf and so never win a minimum.
template <int DPL>
__device__ __forceinline__ void sgm_step(float (&L)[DPL], float& m, const float (&c)[DPL], const bool (&ok)[DPL],
                                         float p1, float p2, float scale) {
  const float lo = dppf<0x138>(L[DPL - 1], kInf);  // wave_shr:1 -- L(d - 1) of this lane's first d
  const float hi = dppf<0x130>(L[0], kInf);        // wave_shl:1 -- L(d + 1) of its last d
  const float mp2 = m + p2;
  float nl[DPL];
  float lm = kInf;
#pragma unroll
  for (int k = 0; k < DPL; ++k) {
    const float a = k == 0 ? lo : L[k - 1];
    const float b = k == DPL - 1 ? hi : L[k + 1];
    const float best = fminf(fminf(L[k], fminf(a, b) + p1), mp2);
    nl[k] = ok[k] ? fmaf(scale, c[k], best - m) : kInf;
    lm = fminf(lm, nl[k]);
  }
#pragma unroll
  for (int k = 0; k < DPL; ++k) L[k] = nl[k];
  m = wave_minf(lm);
}

// Smallest d holding the wave minimum of v (v finite where ok).
template <int DPL>
__device__ __forceinline__ int wave_argmin(const float (&v)[DPL], const bool (&ok)[DPL], int lane) {
  float lm = kInf;
  int kk = DPL;
#pragma unroll
  for (int k = DPL - 1; k >= 0; --k)
    if (ok[k] && v[k] <= lm) {
      lm = v[k];
      kk = k;
    }
  const float gm = wave_minf(lm);
  const uint64_t hit = __ballot(kk < DPL && lm == gm);
  if (hit == 0) return 0;
  const int l0 = __builtin_ctzll(hit);
  return DPL * l0 + __builtin_amdgcn_readlane(kk, l0);
}

// Pixel ring depth: K pixels of cost (and of stored sums) in flight per wave.
template <int DPL>
constexpr int ring_depth() {
  return DPL == 1 ? 16 : (DPL == 2 ? 12 : 8);
}

// Run `count` pixels of one path, starting at pixel p0 and stepping by dp.
// LOADS: add the sum stored at each pixel.  Then either store the result
// (STORES) or write the WTA of it (WTA).
template <int DPL, bool VEC, bool LOADS, bool STORES, bool WTA>
__device__ __forceinline__ void sgm_run(const SgmArgs& a, int p0, int dp, int count, float (&L)[DPL], float& m,
                                        const bool (&ok)[DPL], int lane) {
  constexpr int K = ring_depth<DPL>();
  if (count <= 0) return;
  const int D = a.D;
  const int last = count - 1;
  Slot<DPL, VEC> cb[K], sb[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int pix = p0 + min(j, last) * dp;
    load_slot(cb[j], a.cost + (size_t)pix * D, lane, D);
    if constexpr (LOADS) load_slot(sb[j], a.sum + (size_t)pix * D, lane, D);
  }
  auto body = [&](int i, Slot<DPL, VEC>& c, Slot<DPL, VEC>& s) {
    sgm_step<DPL>(L, m, c.v, ok, a.p1, a.p2, a.scale);
    const int pix = p0 + i * dp;
    float out[DPL];
#pragma unroll
    for (int k = 0; k < DPL; ++k) out[k] = LOADS ? s.v[k] + L[k] : L[k];
    if constexpr (STORES) store_slot<DPL, VEC>(a.sum + (size_t)pix * D, out, lane, D);
    if constexpr (WTA) {
      const int d = wave_argmin<DPL>(out, ok, lane);
      if (lane == 0) a.disp[pix] = d;
    }
  };
  int i0 = 0;
  for (; i0 + K <= count; i0 += K) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      body(i0 + j, cb[j], sb[j]);
      const int pix = p0 + min(i0 + j + K, last) * dp;
      load_slot(cb[j], a.cost + (size_t)pix * D, lane, D);
      if constexpr (LOADS) load_slot(sb[j], a.sum + (size_t)pix * D, lane, D);
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (i0 + j < count) body(i0 + j, cb[j], sb[j]);
}

template <int DPL, bool VEC, bool VERT, bool WTA>
__global__ __launch_bounds__(128) void sgm_line_kernel(SgmArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const bool fwd = threadIdx.x < kWave;
  const int line = blockIdx.x;
  const int n = VERT ? a.H : a.W;
  const int stride = VERT ? a.W : 1;
  const int base = VERT ? line : line * a.W;  // pixel index of the line's first pixel
  const int half = n / 2;                     // wave 0 starts on [0, half), wave 1 on [half, n)
  bool ok[DPL];
  float L[DPL];
#pragma unroll
  for (int k = 0; k < DPL; ++k) {
    ok[k] = DPL * lane + k < a.D;
    L[k] = ok[k] ? 0.0f : kInf;  // with m = 0 the first step gives L = s C
  }
  float m = 0.0f;
  if (fwd)
    sgm_run<DPL, VEC, VERT, true, false>(a, base, stride, half, L, m, ok, lane);
  else
    sgm_run<DPL, VEC, VERT, true, false>(a, base + (n - 1) * stride, -stride, n - half, L, m, ok, lane);
  __syncthreads();  // each half now holds the other wave's contribution
  if (fwd)
    sgm_run<DPL, VEC, true, !WTA, WTA>(a, base + half * stride, stride, n - half, L, m, ok, lane);
  else
    sgm_run<DPL, VEC, true, !WTA, WTA>(a, base + (half - 1) * stride, -stride, half, L, m, ok, lane);
}

template <int DPL, bool VEC>
int run_sgm(const SgmArgs& a, bool vert, bool wta, hipStream_t s) {
  const dim3 block(2 * kWave);
  if (!vert) return launch("sgm_rows", sgm_line_kernel<DPL, VEC, false, false>, dim3(a.H), block, 0, s, a);
  if (!wta) return launch("sgm_cols", sgm_line_kernel<DPL, VEC, true, false>, dim3(a.W), block, 0, s, a);
  return launch("sgm_cols_wta", sgm_line_kernel<DPL, VEC, true, true>, dim3(a.W), block, 0, s, a);
}

}  // namespace

int dispatch_sgm(const SgmArgs& a, bool vert, bool wta, hipStream_t s) {
  const int dpl = (a.D + kWave - 1) / kWave;
  const bool vec = a.D % dpl == 0;
  switch (dpl) {
    case 1: return run_sgm<1, true>(a, vert, wta, s);
    case 2: return vec ? run_sgm<2, true>(a, vert, wta, s) : run_sgm<2, false>(a, vert, wta, s);
    case 3: return run_sgm<3, false>(a, vert, wta, s);
    case 4: return vec ? run_sgm<4, true>(a, vert, wta, s) : run_sgm<4, false>(a, vert, wta, s);
  }
  return fail(ZDT_EUNSUPPORTED, "sgm: max_disp %d > %d", a.D, 4 * kWave);
}

}  // namespace zdt
