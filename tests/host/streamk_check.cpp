// Host check of the stream-K partition used by the library's GEMM launches:
// every (tile, K-tile) iteration of the active tiles is computed exactly once,
// every (tile, segment) partial is written exactly once with seg < the
// tile's segment count, the consumer's segment count matches what was
// written, the writes fit the partial rows the launch code reserves, and the
// XCD-aware range order is a permutation.  Built with g++ (no HIP).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2312_08201_amd/csrc/streamk.h"

using namespace lyap;

static int fails = 0;
#define CHECK(c, ...)                     \
  do {                                    \
    if (!(c)) {                           \
      std::printf("FAIL: " __VA_ARGS__);  \
      std::printf("\n");                  \
      if (++fails > 20) std::exit(1);     \
    }                                     \
  } while (0)

static void check(long long M, int Meff, int ntiles, int grid, int nk, int xcd) {
  const SkPlan p = sk_plan(Meff, ntiles, grid, nk);
  CHECK(p.bm == 32 || p.bm == 64 || p.bm == kGemmBM, "tile height %d", p.bm);
  CHECK((long long)p.mta * p.bm >= Meff && (long long)(p.mta - 1) * p.bm < Meff, "row tiles");
  const int tiles = p.mta * ntiles;
  std::vector<int> cover((size_t)tiles * nk, 0);
  std::vector<int> nseg(tiles, 0), s0v(tiles, 0);
  for (int t = 0; t < tiles; ++t) sk_segments(p, t, s0v[t], nseg[t]);
  std::vector<std::vector<int>> written(tiles);
  for (int t = 0; t < tiles; ++t) written[t].assign(nseg[t], 0);
  const long long rows_avail = sk_part_rows(M, ntiles, grid, nk);
  std::vector<int> seen(grid, 0);
  for (int bid = 0; bid < grid; ++bid) {
    const int v = sk_range_of(bid, grid, xcd);
    CHECK(v >= 0 && v < grid, "range index %d of %d", v, grid);
    seen[v]++;
    long long it, end;
    sk_range(p, v, it, end);
    while (it < end) {
      int t, k0, k1;
      sk_piece(p, it, end, t, k0, k1);
      CHECK(t >= 0 && t < tiles && k0 >= 0 && k1 > k0 && k1 <= nk, "piece t=%d [%d,%d)", t, k0, k1);
      for (int k = k0; k < k1; ++k) cover[(size_t)t * nk + k]++;
      const int seg = v - s0v[t];
      CHECK(seg >= 0 && seg < nseg[t], "seg %d of %d (tile %d)", seg, nseg[t], t);
      if (seg >= 0 && seg < nseg[t]) written[t][seg]++;
      CHECK((long long)(seg + 1) * p.mta * p.bm <= rows_avail,
            "partial rows %lld > %lld (M=%lld Meff=%d grid=%d nk=%d)",
            (long long)(seg + 1) * p.mta * p.bm, rows_avail, M, Meff, grid, nk);
      CHECK((t % p.mta) * p.bm < Meff, "tile row %d beyond the active rows %d", (t % p.mta) * p.bm,
            Meff);
      {
        const int mt = t % p.mta, hb = sk_tile_height(p, mt, Meff);
        const int need = Meff - mt * p.bm < p.bm ? Meff - mt * p.bm : p.bm;
        CHECK(hb >= need && hb <= p.bm && (hb == 32 || hb == 64 || hb == kGemmBM),
              "tile %d height %d for %d rows", mt, hb, need);
      }
      it += k1 - k0;
    }
  }
  for (int v = 0; v < grid; ++v) CHECK(seen[v] == 1, "range %d taken %d times", v, seen[v]);
  for (size_t i = 0; i < cover.size(); ++i)
    CHECK(cover[i] == 1, "iteration %zu covered %d times (Meff=%d grid=%d nk=%d)", i, cover[i],
          Meff, grid, nk);
  for (int t = 0; t < tiles; ++t)
    for (int sg = 0; sg < nseg[t]; ++sg)
      CHECK(written[t][sg] == 1, "tile %d segment %d written %d times", t, sg, written[t][sg]);
}

int main() {
  long long cases = 0;
  const int grids[] = {1, 7, 8, 256, 512, 768, 1024};
  const int nks[] = {1, 3, 16, 24, 48, 96, 256, 512};
  const int nts[] = {1, 3, 32};
  const long long Ms[] = {128, 384, 2304};
  for (long long M : Ms)
    for (int nt : nts)
      for (int nk : nks)
        for (int grid : grids)
          for (int xcd : {0, 1})
            for (int Meff : {1, 9, 32, 33, 64, 65, 127, 128, 129, 300, 1152, 2304}) {
              if (Meff > M) continue;
              check(M, Meff, nt, grid, nk, xcd);
              ++cases;
            }
  if (fails) return 1;
  std::printf("ALL OK (%lld plans)\n", cases);
  return 0;
}
