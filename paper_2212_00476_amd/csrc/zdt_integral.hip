// zdt_integral.hip -- window sums by the paper's Method 2 (Sec. IV-B): the
// integral image of the (border-replicated) image and of its squares, built by
// integrating every row and then every column, and each window sum taken from
// four corners of it.  All arithmetic is uint32 and wraps: the integral of
// I^2 exceeds 2^32 on large images, but a window's sum is below 2^31 and the
// four-corner difference is exact modulo 2^32.
//
// Padded domains (replicated borders, as for every other window sum here):
//   reference  columns -r .. W-1+r            rows -r .. H-1+r
//   target     columns -(D-1)-r .. W-1+r      rows -r .. H-1+r
// An integral array holds (rows+1) x (cols+1) words: row 0 and column 0 are
// zero and entry (i, j) is the sum over padded rows < i and columns < j.
//
//   integral_rows     one workgroup per padded row of both images: inclusive
//                     scan of the row (thread-local runs, a DPP scan over the
//                     wave, wave totals through LDS) for I and I^2
//   integral_cols     64 integral columns per workgroup, the rows split into
//                     16 blocks: block totals, then running sums from offsets
//   integral_windows  one lane per output: four corners per sum
#include "zdt_host.hpp"

namespace zdt {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 12;  // per thread: rows up to 3072 padded columns

// Inclusive scan over the 64 lanes of a wave (uint32, wrapping), by DPP row
// shifts and row broadcasts (lanes without a source add 0).
__device__ __forceinline__ uint32_t wave_scan_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return v;
}

struct IntegralArgs {
  const uint8_t* img[2];  // reference, target
  uint32_t* sum[2];       // integral of I, per image
  uint32_t* sq[2];        // integral of I^2, per image
  int cols[2];            // padded columns per image
  int lead[2];            // padded columns left of column 0: r, and D-1+r
  int pitch, W, H, r;
};

__global__ __launch_bounds__(kScanThreads) void integral_rows_kernel(IntegralArgs a) {
  __shared__ uint32_t wtot[2][kScanThreads / kWave];
  __shared__ uint32_t line[2][kScanThreads * kScanItems];  // the scanned row, for coalesced stores
  const int im = blockIdx.y;
  const int py = blockIdx.x;  // padded row, 0 .. H+2r-1
  const int n = a.cols[im];
  const int y = min(max(py - a.r, 0), a.H - 1);
  const uint8_t* row = a.img[im] + (size_t)y * a.pitch;
  const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
  const int j0 = t * kScanItems;
  uint32_t v[kScanItems], q[kScanItems];
  uint32_t s = 0, s2 = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int j = j0 + i;
    const uint32_t p = j < n ? row[min(max(j - a.lead[im], 0), a.W - 1)] : 0u;
    s += p;
    s2 += p * p;
    v[i] = s;
    q[i] = s2;
  }
  // exclusive offsets of this thread's run: scan of run totals over the block
  const uint32_t is = wave_scan_u32(s), is2 = wave_scan_u32(s2);
  if (lane == kWave - 1) {
    wtot[0][wave] = is;
    wtot[1][wave] = is2;
  }
  __syncthreads();
  uint32_t off = is - s, off2 = is2 - s2;
  for (int w = 0; w < wave; ++w) {
    off += wtot[0][w];
    off2 += wtot[1][w];
  }
  const size_t stride = (size_t)n + 1;
  uint32_t* os = a.sum[im] + (size_t)(py + 1) * stride;
  uint32_t* oq = a.sq[im] + (size_t)(py + 1) * stride;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    line[0][j0 + i] = v[i] + off;
    line[1][j0 + i] = q[i] + off2;
  }
  __syncthreads();
  for (int j = t; j <= n; j += kScanThreads) {
    os[j] = j ? line[0][j - 1] : 0u;
    oq[j] = j ? line[1][j - 1] : 0u;
  }
  if (py == 0)  // the zero row of the integral
    for (int j = t; j <= n; j += kScanThreads) {
      a.sum[im][j] = 0;
      a.sq[im][j] = 0;
    }
}

// Column integration.  grid.x: a strip of 64 integral columns, grid.y: 0/1 =
// sums of image 0/1, 2/3 = squares of image 0/1.  The 16 waves of a workgroup
// split the rows into blocks: each lane first totals its column over its
// block, the totals of the blocks above come through LDS, then the lane
// writes its block's running sums from that offset.
constexpr int kColWaves = 16;
__global__ __launch_bounds__(kWave * kColWaves) void integral_cols_kernel(IntegralArgs a) {
  __shared__ uint32_t tot[kColWaves][kWave];
  const int which = blockIdx.y, im = which & 1;
  const int n = a.cols[im];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int j = blockIdx.x * kWave + lane;
  const bool on = j <= n;
  uint32_t* b = (which < 2 ? a.sum[im] : a.sq[im]) + min(j, n);
  const size_t stride = (size_t)n + 1;
  const int rows = a.H + 2 * a.r;  // integral rows 1 .. rows
  const int per = (rows + kColWaves - 1) / kColWaves;
  const int i0 = 1 + wave * per, i1 = min(i0 + per, rows + 1);
  // 8 rows at a time: the loads of a group are independent and in flight together
  constexpr int G = 8;
  uint32_t s = 0;
  for (int g = i0; g < i1; g += G) {
    uint32_t v[G];
#pragma unroll
    for (int k = 0; k < G; ++k) v[k] = g + k < i1 ? b[(size_t)(g + k) * stride] : 0u;
#pragma unroll
    for (int k = 0; k < G; ++k) s += v[k];
  }
  tot[wave][lane] = s;
  __syncthreads();
  uint32_t acc = 0;
  for (int w = 0; w < wave; ++w) acc += tot[w][lane];
  if (!on) return;
  for (int g = i0; g < i1; g += G) {
    uint32_t v[G];
#pragma unroll
    for (int k = 0; k < G; ++k) v[k] = g + k < i1 ? b[(size_t)(g + k) * stride] : 0u;
#pragma unroll
    for (int k = 0; k < G; ++k)
      if (g + k < i1) {
        acc += v[k];
        b[(size_t)(g + k) * stride] = acc;
      }
  }
}

struct WindowOut {
  int32_t* s[2];   // window sums: reference [H][W], target [H][W+D-1]
  int32_t* ss[2];  // window sums of squares
  int out_cols[2];
};

// grid.y: image; one lane per output pixel of that image
__global__ __launch_bounds__(256) void integral_windows_kernel(IntegralArgs a, WindowOut o) {
  const int im = blockIdx.y;
  const int m = o.out_cols[im];
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)m * a.H) return;
  const int y = (int)(idx / m), x = (int)(idx % m);
  const size_t stride = (size_t)a.cols[im] + 1;
  const int l = 2 * a.r + 1;
  // window rows: padded y .. y+2r (integral rows y and y+l); columns x .. x+2r
  const size_t i0 = (size_t)y * stride, i1 = (size_t)(y + l) * stride;
  const uint32_t* b = a.sum[im];
  const uint32_t* q = a.sq[im];
  if (o.s[im]) o.s[im][idx] = (int32_t)(b[i1 + x + l] - b[i0 + x + l] - b[i1 + x] + b[i0 + x]);
  if (o.ss[im]) o.ss[im][idx] = (int32_t)(q[i1 + x + l] - q[i0 + x + l] - q[i1 + x] + q[i0 + x]);
}

}  // namespace

size_t integral_words(int W, int H, int D, int r, int image) {
  const size_t cols = (size_t)W + 2 * r + (image ? (size_t)D - 1 : 0);
  return ((size_t)H + 2 * r + 1) * (cols + 1);
}

int integral_window_sums(const uint8_t* left, const uint8_t* right, int pitch, int W, int H, int D, int r,
                         int32_t* s_l, int32_t* s_ll, int32_t* s_t, int32_t* s_tt, void* ws, hipStream_t s) {
  IntegralArgs a{};
  a.img[0] = left;
  a.img[1] = right;
  uint32_t* p = (uint32_t*)ws;
  for (int im = 0; im < 2; ++im) {
    const size_t words = integral_words(W, H, D, r, im);
    a.sum[im] = p;
    a.sq[im] = p + words;
    p += 2 * words;
    a.lead[im] = r + (im ? D - 1 : 0);
    a.cols[im] = W + 2 * r + (im ? D - 1 : 0);
  }
  if (a.cols[1] > kScanThreads * kScanItems)
    return fail(ZDT_EUNSUPPORTED, "integral window sums: %d padded columns > %d", a.cols[1],
                kScanThreads * kScanItems);
  a.pitch = pitch;
  a.W = W;
  a.H = H;
  a.r = r;
  int rc = launch("integral_rows", integral_rows_kernel, dim3(H + 2 * r, 2), dim3(kScanThreads), 0, s, a);
  if (rc) return rc;
  rc = launch("integral_cols", integral_cols_kernel, dim3((a.cols[1] + 1 + kWave - 1) / kWave, 4),
              dim3(kWave * kColWaves), 0, s, a);
  if (rc) return rc;
  WindowOut o{{s_l, s_t}, {s_ll, s_tt}, {W, W + D - 1}};
  const long long most = (long long)(W + D - 1) * H;
  return launch("integral_windows", integral_windows_kernel, dim3((unsigned)((most + 255) / 256), 2), dim3(256), 0,
                s, a, o);
}

}  // namespace zdt
