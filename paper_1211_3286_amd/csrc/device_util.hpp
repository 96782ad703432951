// Device helpers shared by the step and adjoint kernels: boundary-aware
// neighbour coordinates, the tile order of the lattice kernels, 32-bit-offset
// loads/stores, pull offsets of the 19 populations, and a block-wide sum of
// five doubles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rlb {
namespace {

__device__ __forceinline__ int nbr(int c, int d, int N, int bc) {
  int s = c + d;
  if (s < 0) s = bc ? 0 : N - 1;
  if (s >= N) s = bc ? N - 1 : 0;
  return s;
}

// Tile order of the fused lattice kernels. The hardware deals workgroups to
// the 8 XCDs round robin (linear id mod 8), and each XCD has its own L2. With
// the plain order the gx tiles of one row (y, z) go to different XCDs, and the
// cache lines they share at their x-boundaries (the pulls from x - 1 and
// x + 1, and the halos of overlapping windows) are fetched from HBM once per
// XCD (measured: 6.7 % over the algorithmic bytes for 128-wide tiles).
// block_tile gives the tiles of a row ids 8 apart, so that one XCD runs the
// whole row, while rows stay spread over the XCDs. Rows in whole groups of 8
// take this order; the remaining rows (fewer than 8) keep the plain order.
// The map from block id to tile is one to one.
__device__ __forceinline__ void block_tile(int& bx, int& by, int& bz) {
  const int gx = gridDim.x, gy = gridDim.y;
  const int h = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int r8 = (gy * (int)gridDim.z) & ~7;  // rows in whole groups of 8
  int row;
  if (gx > 1 && h < gx * r8) {
    const int k = h >> 3;
    bx = k % gx;
    row = (k / gx) * 8 + (h & 7);
  } else {
    bx = h % gx;
    row = h / gx;
  }
  by = row % gy;
  bz = row / gy;
}

// Band order of a 2D grid (gx, gy) with gx a multiple of 8 (else the plain
// order): XCD j runs the band of tile columns [j gx/8, (j+1) gx/8), row by
// row, so that both the x-neighbours (adjacent ids) and the y-neighbours
// (gx/8 ids apart) of a tile share its L2, while the 8 XCDs work in the same
// rows a band apart. One to one.
__device__ __forceinline__ void block_tile_bands(int& bx, int& by) {
  const int gx = gridDim.x;
  bx = blockIdx.x;
  by = blockIdx.y;
  if (gx >= 8 && (gx & 7) == 0) {
    const int h = blockIdx.x + gx * blockIdx.y;
    const int w = gx >> 3;  // tile columns per band
    const int k = h >> 3;   // position in the XCD's sequence
    bx = (h & 7) * w + k % w;
    by = k / w;
  }
}

template <typename T>
__device__ __forceinline__ T ld(const T* plane, uint32_t byteoff) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(plane) + byteoff);
}

template <typename T>
__device__ __forceinline__ void st_nt(T* plane, uint32_t byteoff, T v) {
  __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(plane) + byteoff));
}

template <typename T>
__device__ __forceinline__ void st(T* plane, uint32_t byteoff, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(plane) + byteoff) = v;
}

// Byte offsets of the 19 pull sources of cell (x, y, z) (source = cell - e_a).
__device__ __forceinline__ void pull_offsets(int x, int y, int z, int nx, int ny, int nz, int bcx,
                                             int bcy, int bcz, uint32_t base, uint32_t esz,
                                             uint32_t (&off)[19], uint32_t& self) {
  const int xm = nbr(x, -1, nx, bcx), xp = nbr(x, 1, nx, bcx);
  const int ym = nbr(y, -1, ny, bcy), yp = nbr(y, 1, ny, bcy);
  const int zm = nbr(z, -1, nz, bcz), zp = nbr(z, 1, nz, bcz);
  const uint32_t unx = (uint32_t)nx, uny = (uint32_t)ny;
  const uint32_t r_c = base + ((uint32_t)z * uny + (uint32_t)y) * unx;
  const uint32_t r_ym = base + ((uint32_t)z * uny + (uint32_t)ym) * unx;
  const uint32_t r_yp = base + ((uint32_t)z * uny + (uint32_t)yp) * unx;
  const uint32_t r_zm = base + ((uint32_t)zm * uny + (uint32_t)y) * unx;
  const uint32_t r_zp = base + ((uint32_t)zp * uny + (uint32_t)y) * unx;
  const uint32_t r_ymzm = base + ((uint32_t)zm * uny + (uint32_t)ym) * unx;
  const uint32_t r_ypzp = base + ((uint32_t)zp * uny + (uint32_t)yp) * unx;
  const uint32_t r_ymzp = base + ((uint32_t)zp * uny + (uint32_t)ym) * unx;
  const uint32_t r_ypzm = base + ((uint32_t)zm * uny + (uint32_t)yp) * unx;
  const uint32_t X = (uint32_t)x, XM = (uint32_t)xm, XP = (uint32_t)xp;
  off[0] = (r_c + X) * esz;
  off[1] = (r_c + XM) * esz;
  off[2] = (r_c + XP) * esz;
  off[3] = (r_ym + X) * esz;
  off[4] = (r_yp + X) * esz;
  off[5] = (r_zm + X) * esz;
  off[6] = (r_zp + X) * esz;
  off[7] = (r_ym + XM) * esz;
  off[8] = (r_yp + XP) * esz;
  off[9] = (r_yp + XM) * esz;
  off[10] = (r_ym + XP) * esz;
  off[11] = (r_zm + XM) * esz;
  off[12] = (r_zp + XP) * esz;
  off[13] = (r_zp + XM) * esz;
  off[14] = (r_zm + XP) * esz;
  off[15] = (r_ymzm + X) * esz;
  off[16] = (r_ypzp + X) * esz;
  off[17] = (r_ymzp + X) * esz;
  off[18] = (r_ypzm + X) * esz;
  self = off[0];
}

// Sum five doubles over the block; the result is valid in thread 0.
template <int NT>
__device__ __forceinline__ void block_sum5(double (&v)[5], int tid) {
  __shared__ double sh[(NT + 63) / 64][5];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int i = 0; i < 5; ++i) v[i] += __shfl_xor(v[i], o, 64);
  const int lane = tid & 63, wid = tid >> 6;
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < 5; ++i) sh[wid][i] = v[i];
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      double s = 0.0;
      for (int w = 0; w < (NT + 63) / 64; ++w) s += sh[w][i];
      v[i] = s;
    }
  }
  __syncthreads();
}

}  // namespace
}  // namespace rlb
