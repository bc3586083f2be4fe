// Work order of the molecular-dynamics kernels that gather neighbouring
// links (gauge force, clover force, hopping force, clover build).
//
// Each link or site is read by up to 18 work-items of these kernels.  In
// lexicographic order a site's t-neighbours are a whole t-slice away
// (32^3 sites at 32^3x64, tens of MB of gathered 3x3 matrices), far beyond
// an XCD's 4 MB L2, so the matrices were fetched again for every use.  The
// kernels instead walk the lattice in xy-planes, then z inside a tile of
// 1 << MD_TILE_LG planes, then t, then the next z-tile (t-neighbours are a
// few planes apart), give each XCD one contiguous range of that order, and
// take the four links of 64 sites in four consecutive wavefronts.
#pragma once
#include "qcd_internal.h"

namespace qcd {

constexpr int MD_TILE_LG = 2;

// Site at work position j (0 <= j < V) of the tiled order; returns its
// lexicographic index and its coordinates in y.  A z extent that is not a
// multiple of 1 << MD_TILE_LG takes tiles of 2 planes (every extent is even).
__device__ __forceinline__ int md_site(int j, const Geom& g, int y[4]) {
  const int plane = g.X[0] * g.X[1];
  const int q = j / plane, p = j - q * plane;
  const int tz = g.X[2] % (1 << MD_TILE_LG) == 0 ? MD_TILE_LG : 1;
  const int zi = q & ((1 << tz) - 1), r = q >> tz;
  const int zt = r / g.X[3];
  y[3] = r - zt * g.X[3];
  y[2] = (zt << tz) + zi;
  y[1] = p / g.X[0];
  y[0] = p - y[1] * g.X[0];
  return lex(y, g);
}

// Work position of this work-item in a per-site launch (XCD-contiguous).
__device__ __forceinline__ int md_position() {
  return xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}

// Link of this work-item in a per-link launch of 64-wide workgroups over
// 4 * ceil(V / 64) workgroups: workgroup b takes direction b % 4 of the
// sites 64 (b / 4) ... 64 (b / 4) + 63 of the tiled order, so that the four
// directions of a site run in consecutive workgroups of one XCD and every
// wavefront has one direction.  Returns false past the lattice.  mu is
// derived from the work-item index rather than from the workgroup index:
// with a workgroup-uniform mu the compiler restructures the clover force's
// plane loop (more accumulator-register traffic) and that kernel took 20 %
// longer at 32^3x64.
__device__ __forceinline__ bool md_link(const Geom& g, int& mu, int& i, int y[4]) {
  const int t = xcd_block(blockIdx.x, gridDim.x) * 64 + threadIdx.x;
  mu = (t >> 6) & 3;
  const int j = ((t >> 8) << 6) | (t & 63);
  if (j >= g.V) return false;
  i = md_site(j, g, y);
  return true;
}
inline int md_link_blocks(const Geom& g) { return 4 * ((g.V + 63) / 64); }

}  // namespace qcd
