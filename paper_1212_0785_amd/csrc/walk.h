// Walk of the site-blocked link kernels: which parity and checkerboard
// site a work-item of the staple force, the plaquette sum or the fermion
// force takes.
#pragma once

#include "device.h"

namespace hmc {

// A walk unit is a 64-site chunk of one parity; consecutive units
// alternate the parities.  Where the lattice admits the Dslash's tiled
// order (tiled != 0), XCD x (blocks with blockIdx.x % 8 == x) takes units
// 0, 1, ... of its own t-slices in that order: y-blocks of kGfYBlock chunks
// (or whole z-planes), or, where a z-plane is not a whole number of chunks,
// the chunks of the t-slices, t-slice fastest (dslash_site in device.h).
// Otherwise unit u covers chunk u / 2 of parity u % 2, u from XCD-contiguous
// block ranges.  The links a site's staples or plaquettes share with its
// neighbours' are then fetched into L1 / L2 once for all four directions
// and both parities, where a parity-major or direction-major sweep finds
// the +-z and +-t neighbours long evicted.  *s may be >= Vh in the linear
// walk (ragged last chunk).
constexpr int kGfYBlock = 2;

__device__ __forceinline__ void walk_site(const Lat& g, int xcd, int u, int* par, int* s) {
  const int lane = threadIdx.x & 63;
  *par = u & 1;
  const int w = u >> 1;  // 64-site chunk, in walk order
  if (g.tiled && g.tile_y == 0) {  // chunks of the t-slices, t-slice fastest
    *s = (xcd * g.tile_t + w % g.tile_t) * g.slice + (w / g.tile_t) * 64 + lane;
  } else if (g.tiled) {
    const int c = w % g.tile_y, q = w / g.tile_y;
    const int t = xcd * g.tile_t + q % g.tile_t, q2 = q / g.tile_t;
    const int z = q2 % g.L[2], yb = q2 / g.L[2];
    *s = t * g.slice + z * g.plane + (yb * g.tile_y + c) * 64 + lane;
  } else {
    *s = w * 64 + lane;
  }
}

// The XCD-local (tiled) or global (linear) walk unit of block b scaled by
// `per`, the units per block.
__device__ __forceinline__ int walk_unit(const Lat& g, int per) {
  if (g.tiled) return (blockIdx.x >> 3) * per;
  return xcd_remap(blockIdx.x, gridDim.x) * per;
}

// Lattice argument of the site-blocked walk (tiled where admitted).
inline Lat walk_lat(const LatArg& g) {
  Lat lat = to_lat(g);
  if (tiled_order_valid(g)) {
    lat.tiled = 1;
    lat.plane = g.L[0] * g.L[1] / 2;
    lat.slice = lat.plane * g.L[2];
    lat.tile_r = lat.plane % 64 == 0 ? lat.plane / 64 : 0;
    lat.tile_t = g.L[3] / 8;
    // y-blocks of kGfYBlock chunks, else whole planes, else (tile_r = 0) t-slice chunks
    lat.tile_y = lat.tile_r == 0 ? 0 : lat.tile_r % kGfYBlock == 0 ? kGfYBlock : lat.tile_r;
  }
  return lat;
}

}  // namespace hmc
