// Host emulation of the V-pass WTA butterfly (zdt_device.hpp): random keys
// go through the six merge stages with the lane semantics of the gfx950
// instructions (permlane32/permlane16 swaps as documented for gfx950 and
// checked on the device; DPP row_ror:8, row_half_mirror, quad_perm xor 2 and
// xor 1), then the lane that bfly_map() names must hold each pixel's minimum
// over all 64 lanes.  Runs on the host only.
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <vector>
#include <algorithm>
#include "zdt_device.hpp"
using namespace zdt;
typedef std::vector<uint32_t> Reg;
static Reg dpp(const Reg& a, int st) {
  Reg o(64);
  for (int l = 0; l < 64; ++l) {
    int src;
    if (st == 3) src = (l & ~15) | ((l + 8) & 15);
    else if (st == 4) src = (l & ~7) | (7 - (l & 7));
    else if (st == 5) src = l ^ 2;
    else src = l ^ 1;
    o[l] = std::min(a[l], a[src]);
  }
  return o;
}
template <int N>
int check(unsigned seed) {
  srand(seed);
  std::vector<Reg> r(N, Reg(64)), u;
  for (auto& x : r) for (auto& v : x) v = rand() % 50;
  u = r;
  int n = N;
  for (int st = 1; st <= 6; ++st) {
    const int m = (n + 1) / 2;
    std::vector<Reg> y(m, Reg(64));
    for (int i = 0; i < m; ++i) {
      const Reg& A = r[2 * i];
      const bool pair = 2 * i + 1 < n;
      const Reg& B = pair ? r[2 * i + 1] : A;
      if (st <= 2) {
        Reg f(64), g(64);
        for (int l = 0; l < 64; ++l) {
          if (st == 1) { f[l] = l < 32 ? A[l] : B[l - 32]; g[l] = l < 32 ? A[l + 32] : B[l]; }
          else {
            const int row = l / 16, j = l % 16;
            const int rows_f[4][2] = {{0, 0}, {1, 0}, {0, 2}, {1, 2}};  // (operand, row) of first
            const int rows_g[4][2] = {{0, 1}, {1, 1}, {0, 3}, {1, 3}};
            f[l] = (rows_f[row][0] ? B : A)[rows_f[row][1] * 16 + j];
            g[l] = (rows_g[row][0] ? B : A)[rows_g[row][1] * 16 + j];
          }
        }
        for (int l = 0; l < 64; ++l) y[i][l] = std::min(f[l], g[l]);
      } else {
        const int span = 32 >> (st - 2), half = span / 2;
        Reg ma = dpp(A, st), mb = dpp(B, st);
        for (int l = 0; l < 64; ++l) y[i][l] = pair ? ((l % span) < half ? ma[l] : mb[l]) : ma[l];
      }
    }
    r = y;
    n = m;
  }
  constexpr BflyMap<N> map = bfly_map<N>();
  int bad = 0;
  for (int k = 0; k < N; ++k) {
    const uint32_t want = *std::min_element(u[k].begin(), u[k].end());
    if (map.reg[k] < 0 || r[map.reg[k]][map.lane[k]] != want) ++bad;
  }
  return bad;
}
int main() {
  int bad = 0;
  for (unsigned s = 0; s < 20; ++s)
    bad += check<8>(s) + check<12>(s) + check<24>(s) + check<36>(s) + check<48>(s) + check<72>(s) + check<1>(s) +
           check<3>(s) + check<65>(s);
  printf("bad %d\n", bad);
  return bad != 0;
}
