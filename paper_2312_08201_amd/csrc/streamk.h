// Stream-K partition of the library's dynamic-M GEMM launches: plain C++
// shared by the GEMM kernels, their consumers and the host launch code (and
// compiled on its own by the host-side tests).
#pragma once

#if defined(__HIPCC__)
#define LYAP_HD __host__ __device__
#else
#define LYAP_HD
#endif

namespace lyap {

constexpr int kGemmBM = 128;
constexpr int kGemmBN = 128;

// Stream-K plan of a dynamic-M GEMM launch.  The (tile, K-tile) iterations
// of the active row tiles, tile-major with tile t = nt * mta + mt, are cut
// into consecutive ranges of `per` iterations, one range per workgroup, so
// that every workgroup of the grid carries the same share whatever the
// number of active rows (a one-tile-per-workgroup launch leaves the last
// wave of tiles on a fraction of the CUs).  A workgroup writes each piece of
// a tile it computed to partial buffer seg = (its range index) - (index of
// the first range touching the tile); the consumer adds a tile's segments in
// segment order, so the sum is deterministic for a given active row count.
// A range holds at least kSkMinIters K-tiles (or the whole K), which bounds
// the segments per tile and the partial traffic.  Same formulas on host and
// device.
//
// Tile height: few active rows (a sweep's tail) take 32- or 64-row tiles, so
// that the MFMA work follows the active rows instead of a padded 128-row
// tile; every tile streams the whole B panel, so taller tiles are kept
// beyond 64 rows.
constexpr int kSkMinIters = 16;
struct SkPlan {
  int bm, mta, ntiles, nk, per;
};
LYAP_HD inline int sk_tile_rows(int Meff) { return Meff <= 32 ? 32 : (Meff <= 64 ? 64 : kGemmBM); }
LYAP_HD inline SkPlan sk_plan(int Meff, int ntiles, int grid, int nk) {
  SkPlan p;
  p.bm = sk_tile_rows(Meff);
  p.mta = (Meff + p.bm - 1) / p.bm;
  p.ntiles = ntiles;
  p.nk = nk;
  const long long total = (long long)p.mta * ntiles * nk;
  long long per = grid > 0 ? (total + grid - 1) / grid : total;
  const int lo = nk < kSkMinIters ? nk : kSkMinIters;
  if (per < lo) per = lo;
  if (per < 1) per = 1;
  p.per = (int)per;
  return p;
}
// index of the first range touching tile t, and the number of ranges that do
LYAP_HD inline void sk_segments(const SkPlan& p, int t, int& s0, int& ns) {
  const long long a = (long long)t * p.nk;
  s0 = (int)(a / p.per);
  ns = (int)((a + p.nk - 1) / p.per) - s0 + 1;
}
// Rows computed for row tile mt: bm, except that the last row tile of a
// 128-row plan takes 32 or 64 rows when the active rows end within them (the
// partial layout keeps the bm-row stride, so consumers are unaffected).
LYAP_HD inline int sk_tile_height(const SkPlan& p, int mt, int Meff) {
  if (p.bm != kGemmBM || mt < p.mta - 1) return p.bm;
  const int rem = Meff - mt * p.bm;
  return rem <= 32 ? 32 : (rem <= 64 ? 64 : kGemmBM);
}
// the iteration range [first, end) of range index v
LYAP_HD inline void sk_range(const SkPlan& p, int v, long long& first, long long& end) {
  const long long total = (long long)p.mta * p.ntiles * p.nk;
  first = (long long)v * p.per;
  end = first + p.per < total ? first + p.per : total;
}
// the piece of the range starting at iteration it: tile t, K-tiles [k0, k1);
// the next piece starts at it + (k1 - k0)
LYAP_HD inline void sk_piece(const SkPlan& p, long long it, long long end, int& t, int& k0,
                             int& k1) {
  t = (int)(it / p.nk);
  k0 = (int)(it - (long long)t * p.nk);
  const long long left = end - it;
  k1 = left < p.nk - k0 ? k0 + (int)left : p.nk;
}
// rows (of ldc elements) of partials a stream-K launch of `grid` workgroups
// may write for any active row count up to M: segments are stored
// seg-major, mta * bm rows each, and a tile has at most
// ceil((nk - 1) / per) + 1 of them.  The plan depends on the active rows
// through bm and mta only, so one row count per (bm, mta) is checked.
inline long long sk_part_rows(long long M, int ntiles, int grid, int nk) {
  long long rows = 0;
  auto upd = [&](int Meff) {
    const SkPlan p = sk_plan(Meff, ntiles, grid, nk);
    const long long ns = (nk - 1 + p.per - 1) / p.per + 1;
    if (ns * p.mta * p.bm > rows) rows = ns * p.mta * p.bm;
  };
  if (M >= 1) upd(1);
  if (M > 32) upd(33);
  if (M > 64) {
    const int mtiles = (int)((M + kGemmBM - 1) / kGemmBM);
    for (int mta = 1; mta <= mtiles; ++mta) upd(mta * kGemmBM);
  }
  return rows;
}

// Range index of workgroup bid in a stream-K launch of `grid` workgroups.
// With the XCD-aware order the workgroups of one XCD (dispatched round-robin,
// bid % 8) take consecutive ranges, so the tiles of one B column panel stay
// in that XCD's L2.  A permutation of [0, grid).
LYAP_HD inline int sk_range_of(int bid, int grid, int xcd) {
  if (xcd && grid % 8 == 0) return (bid % 8) * (grid / 8) + bid / 8;
  return bid;
}

}  // namespace lyap
