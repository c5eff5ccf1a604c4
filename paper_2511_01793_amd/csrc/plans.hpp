// Shape variants the kernels are instantiated for, shared by device and host
// code.  The autotuner in api.hip times them on the caller's data and picks
// one per context.
//
// FFT plan (m, variant): the 1-D length-m transform is split as m = R1 * R2
// (pass 1: R2-point DFTs over stride-R1 elements, pass 2: R1-point DFTs over
// contiguous runs), computed by NT threads per patch.  Each thread owns
// m^2 / (4 NT) 2 x 2 pixel blocks in the per-pixel phases.  Variant 0 is the
// default.  Plans with the same (R1, R2) give bitwise-identical results;
// another split reorders the DFT arithmetic (same transform, other rounding)
// and lays the intensities out in its own transform order.
//
// XL = 1: the patch kernel keeps the tile in registers through the two passes
// of each dimension and transposes a line's 8 lanes with cross-lane moves, so
// the tile goes through LDS between the row and the column phase instead of
// after every pass (m = 64, 8 * 8 split, 1024 threads only).  The plan's other
// kernels use the LDS passes.  The arithmetic is the same either way, so the
// results are bitwise those of the other plans with the same split.
// DG = 1: the patch kernel gathers the exit wave straight into the registers of
// the first (strided) row pass, item (row, g) of that pass loading its own points,
// so the pass needs no LDS round trip and no barrier of its own.  The pass's
// arithmetic is unchanged, so the results are bitwise those of DG = 0.  (Plan
// (128, 1) with it needs 15 twiddles per thread and spills: measured slower.)
// AMP is where the patch kernel issues the loads of the measured intensities:
// 0 with the exit-wave loads at the start, k > 0 after the k-th forward pass.
// Plans whose registers are tight at 1024 threads issue them late, so the
// values are not held through the passes before (they would be spilled).
//
// Finalize shape (variant): FNT threads per work item, object tiles of
// T x T pixels, and the order the blocks take the tiles in.  Every shape sums
// the same terms in the same order, so the results are bitwise identical; only
// the speed differs.
#pragma once

namespace emg {

template <int M, int V> struct Plan;
template <> struct Plan<32, 0> { static constexpr int R1 = 8, R2 = 4, NT = 256; static constexpr int AMP = 0, XL = 0, DG = 0; };
template <> struct Plan<32, 1> { static constexpr int R1 = 4, R2 = 8, NT = 256; static constexpr int AMP = 0, XL = 0, DG = 0; };
template <> struct Plan<64, 0> { static constexpr int R1 = 8, R2 = 8, NT = 1024; static constexpr int AMP = 0, XL = 0, DG = 0; };
template <> struct Plan<64, 1> { static constexpr int R1 = 16, R2 = 4, NT = 1024; static constexpr int AMP = 2, XL = 0, DG = 0; };
template <> struct Plan<64, 2> { static constexpr int R1 = 4, R2 = 16, NT = 1024; static constexpr int AMP = 0, XL = 0, DG = 0; };
template <> struct Plan<64, 3> { static constexpr int R1 = 8, R2 = 8, NT = 1024; static constexpr int AMP = 0, XL = 1, DG = 0; };
template <> struct Plan<128, 0> { static constexpr int R1 = 16, R2 = 8, NT = 1024; static constexpr int AMP = 3, XL = 0, DG = 1; };
template <> struct Plan<128, 1> { static constexpr int R1 = 8, R2 = 16, NT = 1024; static constexpr int AMP = 2, XL = 0, DG = 0; };
template <> struct Plan<128, 2> { static constexpr int R1 = 16, R2 = 8, NT = 512; static constexpr int AMP = 0, XL = 0, DG = 0; };
// m = 256: the tile exceeds LDS; strips of 16 lines per workgroup (kernels_m256.hip)
template <> struct Plan<256, 0> { static constexpr int R1 = 16, R2 = 16, NT = 256; static constexpr int AMP = 0, XL = 0, DG = 0; };

template <int M> struct PlanCount;
template <> struct PlanCount<32> { static constexpr int value = 2; };
template <> struct PlanCount<64> { static constexpr int value = 4; };
template <> struct PlanCount<128> { static constexpr int value = 3; };
template <> struct PlanCount<256> { static constexpr int value = 1; };

constexpr int kMaxFftPlans = 4;

// host-side description of FFT plan (m, v); false if there is no such plan
inline bool fft_plan_desc(int m, int v, int* r1, int* r2, int* nt) {
  struct D {
    int m, v, r1, r2, nt;
  };
  static const D t[] = {{32, 0, 8, 4, 256},   {32, 1, 4, 8, 256},   {64, 0, 8, 8, 1024},
                        {64, 1, 16, 4, 1024}, {64, 2, 4, 16, 1024}, {64, 3, 8, 8, 1024},
                        {128, 0, 16, 8, 1024}, {128, 1, 8, 16, 1024}, {128, 2, 16, 8, 512},
                        {256, 0, 16, 16, 256}};
  for (const D& d : t)
    if (d.m == m && d.v == v) {
      *r1 = d.r1;
      *r2 = d.r2;
      *nt = d.nt;
      return true;
    }
  return false;
}
inline int fft_plan_count(int m) { return m == 32 ? 2 : m == 64 ? 4 : m == 128 ? 3 : m == 256 ? 1 : 0; }

// finalize shapes: (threads per item, object tile side) for F & 3, and the
// order in which the grid's blocks take the object tiles for F >> 2: row-major
// (0), banded (1) or rows per XCD (2).  Block i of a launch runs on XCD
// i mod kDispatchXcds.
//  * banded: XCD x takes the x-th contiguous band of tile rows, the band of the
//    object whose patches the same XCD ran when the minibatch was listed for the
//    XCDs, so their numerators may still be in its L2;
//  * rows per XCD: XCD x takes the tile rows x, x + 8, x + 16, ...: the tiles side
//    by side in a row share the cache lines where a numerator row segment crosses
//    from one tile into the next, and those lines are then fetched into one L2
//    instead of two.
// Which order is faster depends on how the scan spreads the work (uniform rasters
// favour bands, a dense centre favours row-major or rows per XCD), so all are
// candidates for the autotuner.  The order changes no result.
constexpr int kDispatchXcds = 8;
template <int F> struct FinShapeBase;
template <> struct FinShapeBase<0> { static constexpr int FNT = 256, T = 32; };
template <> struct FinShapeBase<1> { static constexpr int FNT = 256, T = 16; };
template <> struct FinShapeBase<2> { static constexpr int FNT = 512, T = 32; };
template <> struct FinShapeBase<3> { static constexpr int FNT = 1024, T = 64; };
template <int F> struct FinShape : FinShapeBase<F & 3> {
  static constexpr int ORDER = F >> 2;  // 0 row-major, 1 banded, 2 rows per XCD
  static constexpr bool BANDED = ORDER == 1;
};
constexpr int kFinShapes = 12;

inline bool fin_shape_desc(int f, int* fnt, int* tile, int* order = nullptr) {
  static const int t[4][2] = {{256, 32}, {256, 16}, {512, 32}, {1024, 64}};
  if (f < 0 || f >= kFinShapes) return false;
  *fnt = t[f & 3][0];
  *tile = t[f & 3][1];
  if (order) *order = f >> 2;
  return true;
}

// Tile taken by block i < ntiles in the rows-per-XCD order (tpr tiles per tile row).
// Blocks are listed XCD by XCD (block i is the (i / X)-th of XCD i mod X) and tiles
// rows x, x + X, ... for x = 0, 1, ...; the i-th block in the first list takes the
// tile at the same place in the second.  A bijection of [0, ntiles) for any sizes.
__host__ __device__ inline int rows_per_xcd_tile(int i, int ntiles, int tpr) {
  constexpr int X = kDispatchXcds;
  const int x = i % X, trows = ntiles / tpr;
  int pos = i / X;
  for (int y = 0; y < x; ++y) pos += (ntiles - y + X - 1) / X;  // blocks on the XCDs before x
  for (int y = 0; y < X; ++y) {
    const int seg = ((trows - y + X - 1) / X) * tpr;  // tiles in the rows y, y + X, ...
    if (pos < seg) return (y + X * (pos / tpr)) * tpr + pos % tpr;
    pos -= seg;
  }
  return i;  // not reached for i < ntiles
}

// Slot groups of the probe sums in the finalize: each probe pixel's sum over
// the minibatch is split into G contiguous slot ranges added in parallel, then
// combined in group order.  G depends only on the configured minibatch size,
// so every path and finalize shape sums in the same order.
inline int probe_groups(int minibatch) { return minibatch >= 64 ? 16 : (minibatch >= 16 ? 8 : 4); }

}  // namespace emg
