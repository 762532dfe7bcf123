// Uniform cell grid over the sphere centres, used by the two neighbour searches of the solver (the
// pair lists of the near-field preconditioner and the 16 nearest neighbours behind the warm-start
// features). Cell keys are Morton codes of the integer cell coordinates, so one radix sort by key
// puts every cell's spheres next to each other (in index order: the sort is stable) and keeps
// neighbouring cells close in memory. The cell size and counts are chosen on the device from the
// bounding box, so a build needs no host round trip.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace mbs {

constexpr int kGridAxisBits = 10;  // at most 1024 cells per axis (30-bit keys)

struct GridHdr {
  double lo[3];  // lower corner of the bounding box
  double h;      // cell edge
  double inv_h;
  int g[3];      // cells per axis
  int maxocc;    // most spheres in one cell
  int n;         // spheres
  int pad;
};

// Read-only view of a built grid (device pointers).
struct GridView {
  const GridHdr* hdr;
  const double* Rs;      // [n][4] centres in sorted order (x, y, z, unused)
  const int32_t* perm;   // [n] sphere index at each sorted position
  const int32_t* start;  // [cells] first sorted position of each cell
  const int32_t* end;    // [cells] one past the last (start == end: empty cell)
  int n;
};

__device__ __forceinline__ int grid_cell1(double x, double lo, double inv_h, int g) {
  const int c = (int)floor((x - lo) * inv_h);
  return min(max(c, 0), g - 1);
}

__device__ __forceinline__ int grid_linear(const GridHdr& H, int x, int y, int z) {
  return (z * H.g[1] + y) * H.g[0] + x;
}

// A grid is crowded when it has few cells or one cell holds at least 1/8 of all spheres (a
// collapsed cluster): a sphere's 27 cells then hold a large share of all spheres, and an all-pairs
// scan through LDS beats walking the cells. The searches launch both variants and each returns at
// once unless the grid (read on the device) is of its kind.
constexpr int kDenseCells = 128;

__device__ __forceinline__ bool grid_dense(const GridHdr* hdr) {
  return (int64_t)hdr->g[0] * hdr->g[1] * hdr->g[2] < kDenseCells || 8 * (int64_t)hdr->maxocc >= hdr->n;
}

// Workspace bytes for a grid of n centres and at most max_cells cells.
size_t grid_ws_bytes(int n, int64_t max_cells);
// Build the grid of R [n x 3] with cell edge >= h_min and at most max_cells cells; ws is device
// memory of grid_ws_bytes(n, max_cells) bytes (256-byte aligned). Returns a HIP error code.
hipError_t grid_build(const double* R, int n, double h_min, int64_t max_cells, void* ws,
                      size_t ws_bytes, GridView* view, hipStream_t s);
// The same for the centres of a periodic cubic box of side L: nc cells of edge L / nc per axis from
// the origin (nc <= 1024), every centre wrapped into [0, L) first (Rs holds the wrapped centres);
// ws: grid_ws_bytes(n, nc^3) bytes.
hipError_t grid_build_box(const double* R, int n, double L, int nc, void* ws, size_t ws_bytes,
                          GridView* view, hipStream_t s);

}  // namespace mbs
