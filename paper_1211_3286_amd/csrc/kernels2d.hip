// Kernels of the D2Q9 MRT model (Sec. V.A) for gfx950.
//
// Population storage (one buffer): 18 planes of cs elements, planes 0..8 hold
// f_a and planes 9..17 hold g_a (D2Q9 velocity order of rlb.h). Two buffers
// alternate (A/B), as for D3Q19. The fused step reads 18 values per cell,
// collides in registers (cell2d.hpp) and writes 18: 2 x 18 x sizeof(T) bytes
// of HBM traffic per cell update.

#include <hip/hip_runtime.h>

#include "cell2d.hpp"
#include "device_util.hpp"
#include "internal.hpp"

namespace rlb {

namespace {

// Fields of the y - 1 and y + 1 neighbours of cell (x, y) for the correction
// term (their pulled g, recovered), neighbours picked by the y-streaming rule.
template <typename T>
__device__ __forceinline__ void c7_neighbours(const T* __restrict__ src, int64_t cs, int x,
                                              int y, int nx, int ny, int bcx, int bcy,
                                              uint32_t base, const Ref& ref,
                                              d2q9::C7Fields& fm, d2q9::C7Fields& fp) {
  uint32_t off[9], self;
  d2q9::pull_offsets(x, nbr(y, -1, ny, bcy), nx, ny, bcx, bcy, base, sizeof(T), off, self);
  fm = d2q9::c7_fields_at(src, cs, off, ref);
  d2q9::pull_offsets(x, nbr(y, 1, ny, bcy), nx, ny, bcx, bcy, base, sizeof(T), off, self);
  fp = d2q9::c7_fields_at(src, cs, off, ref);
}

// -------------------------------------------------------------------------
// Fused step on one nx x ny lattice: grid (ceil(nx/BX), ceil(ny/(BY*CY))),
// block (BX, BY); each thread updates CY cells along y. Tiles are taken in
// the band order of block_tile_bands (the rows a tile pulls from above and
// below, and the lines it shares with its x-neighbours, are L2 hits: 1.02x
// the algorithmic bytes instead of 1.04-1.17x). With CORR the plain order
// measured slightly faster (0.47-0.49 against 0.49 ms per 4096^2 FP32 step),
// although it moves more bytes, and is kept. CORR adds the
// correction of Eqs. (37)-(38) (each cell recovers its two y-neighbours from
// their pulled populations: 18 more loads, mostly L2 hits). NTS: nontemporal
// stores, as in k_step_lattice.
// -------------------------------------------------------------------------
template <typename T, int BX, int BY, int CY, bool DIAG, bool CORR, bool EXT, bool NTS>
__global__ __launch_bounds__(BX* BY) void k_d2q9_lattice(const T* __restrict__ src,
                                                        T* __restrict__ dst, LatticeGeom geo,
                                                        double* __restrict__ partials,
                                                        unsigned long long* __restrict__ bad) {
  int bx = blockIdx.x, by = blockIdx.y;
  if constexpr (!CORR) block_tile_bands(bx, by);
  const int x = bx * BX + threadIdx.x;
  const int tid = threadIdx.y * BX + threadIdx.x;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int nbad = 0;
  const uint32_t esz = sizeof(T);
#pragma unroll 1
  for (int k = 0; k < CY; ++k) {
    const int y = (by * CY + k) * BY + threadIdx.y;
    if (x < geo.nx && y < geo.ny) {
      d2q9::C7Fields fm, fp;
      if constexpr (CORR)
        c7_neighbours(src, geo.cs, x, y, geo.nx, geo.ny, geo.bcx, geo.bcy, 0u, geo.ref, fm,
                      fp);
      uint32_t off[9], self;
      d2q9::pull_offsets(x, y, geo.nx, geo.ny, geo.bcx, geo.bcy, 0u, esz, off, self);
      T f[9], g[9];
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        f[a] = ld(src + (int64_t)a * geo.cs, off[a]);
        g[a] = ld(src + (int64_t)(9 + a) * geo.cs, off[a]);
      }
      Sums s;
      const bool ok =
          d2q9::collide<T, CORR, EXT>(f, g, geo.rt, geo.ref, s, &fm, &fp, &geo.ext);
      nbad += ok ? 0 : 1;
      if (DIAG)
#pragma unroll
        for (int i = 0; i < 5; ++i) acc[i] += s.v[i];
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        if constexpr (NTS) {
          st_nt(dst + (int64_t)a * geo.cs, self, f[a]);
          st_nt(dst + (int64_t)(9 + a) * geo.cs, self, g[a]);
        } else {
          st(dst + (int64_t)a * geo.cs, self, f[a]);
          st(dst + (int64_t)(9 + a) * geo.cs, self, g[a]);
        }
      }
    }
  }
  if (nbad) count_bad(bad, nbad);
  if (DIAG) {
    block_sum5<BX * BY>(acc, tid);
    if (tid == 0) {
      const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
      for (int i = 0; i < 5; ++i) partials[b * 5 + i] = acc[i];
    }
  }
}

// -------------------------------------------------------------------------
// The same step with the correction term, the C_7 fields shared through LDS:
// grid (ceil(nx/BX), ceil(ny/BY)), block (BX, BY), one cell per thread. Each
// thread recovers the fields of its own cell from its pulled g and publishes
// them, keeping the recovery for its own collision; the block's first and
// last valid rows also recover the rows beyond (their y-neighbours by the
// y-streaming rule). A cell so costs 1 + 2/BY recoveries instead of the 3 of
// k_d2q9_lattice with the correction, whose step is VALU-bound. Tiles are
// taken in the band order of block_tile_bands (the halo rows and the lines
// shared with x-neighbours are L2 hits: 1.02x the algorithmic bytes instead of
// 1.09-1.20x). Results are those of k_d2q9_lattice bit for bit (the same
// fields from the same pulled g).
// -------------------------------------------------------------------------
template <typename T, int BX, int BY, bool DIAG, bool EXT, bool NTS>
__global__ __launch_bounds__(BX* BY) void k_d2q9_lattice_c7(const T* __restrict__ src,
                                                           T* __restrict__ dst, LatticeGeom geo,
                                                           double* __restrict__ partials,
                                                           unsigned long long* __restrict__ bad) {
  constexpr int R = BY + 2;  // LDS rows: the row above, BY rows, the row below
  __shared__ double cf[4][R * BX];
  __shared__ int cok[R * BX];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * BX + tx;
  int bx = blockIdx.x, by = blockIdx.y;
  block_tile_bands(bx, by);
  const int x = bx * BX + tx;
  const int y0 = by * BY;
  const int rows = min(BY, geo.ny - y0);  // valid rows of the block (the grid makes it >= 1)
  const int y = y0 + ty;
  const bool xin = x < geo.nx;
  const bool in = xin && ty < rows;
  const uint32_t esz = sizeof(T);
  auto publish = [&](int slot, const d2q9::C7Fields& F) {
    cf[0][slot] = F.x1;
    cf[1][slot] = F.gam;
    cf[2][slot] = F.su2;
    cf[3][slot] = F.su;
    cok[slot] = F.ok ? 1 : 0;
  };
  T f[9], g[9];
  uint32_t self = 0;
  d2q9::Recovered rec;
  if (in) {
    uint32_t off[9];
    d2q9::pull_offsets(x, y, geo.nx, geo.ny, geo.bcx, geo.bcy, 0u, esz, off, self);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      f[a] = ld(src + (int64_t)a * geo.cs, off[a]);
      g[a] = ld(src + (int64_t)(9 + a) * geo.cs, off[a]);
    }
    // the cell's own recovery serves both its published fields and its
    // collision (the correction needs the paper's equation of state, for which
    // the recovery is that of c7_fields_of)
    rec = d2q9::recovered<T, EXT>(f, g, geo.ref, &geo.ext);
    publish((ty + 1) * BX + tx, d2q9::c7_fields(rec.mac, rec.ok));
  }
  if (xin && ty == 0) {  // the y-neighbour below the first row: LDS row 0
    uint32_t off[9], s0;
    d2q9::pull_offsets(x, nbr(y0, -1, geo.ny, geo.bcy), geo.nx, geo.ny, geo.bcx, geo.bcy, 0u,
                       esz, off, s0);
    publish(tx, d2q9::c7_fields_at(src, geo.cs, off, geo.ref));
  }
  if (xin && ty == rows - 1) {  // the y-neighbour above the last row: LDS row rows + 1
    uint32_t off[9], s1;
    d2q9::pull_offsets(x, nbr(y0 + rows - 1, 1, geo.ny, geo.bcy), geo.nx, geo.ny, geo.bcx,
                       geo.bcy, 0u, esz, off, s1);
    publish((rows + 1) * BX + tx, d2q9::c7_fields_at(src, geo.cs, off, geo.ref));
  }
  __syncthreads();
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int nbad = 0;
  if (in) {
    const int m = ty * BX + tx, p = (ty + 2) * BX + tx;
    const d2q9::C7Fields fm{cf[0][m], cf[1][m], cf[2][m], cf[3][m], cok[m] != 0};
    const d2q9::C7Fields fp{cf[0][p], cf[1][p], cf[2][p], cf[3][p], cok[p] != 0};
    Sums s;
    const bool ok = d2q9::collide_recovered<T, true, EXT>(f, g, rec, geo.rt, geo.ref, s, &fm,
                                                          &fp, &geo.ext);
    nbad += ok ? 0 : 1;
    if (DIAG)
#pragma unroll
      for (int i = 0; i < 5; ++i) acc[i] += s.v[i];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      if constexpr (NTS) {
        st_nt(dst + (int64_t)a * geo.cs, self, f[a]);
        st_nt(dst + (int64_t)(9 + a) * geo.cs, self, g[a]);
      } else {
        st(dst + (int64_t)a * geo.cs, self, f[a]);
        st(dst + (int64_t)(9 + a) * geo.cs, self, g[a]);
      }
    }
  }
  if (nbad) count_bad(bad, nbad);
  if (DIAG) {
    block_sum5<BX * BY>(acc, tid);
    if (tid == 0) {
      const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
      for (int i = 0; i < 5; ++i) partials[b * 5 + i] = acc[i];
    }
  }
}

// -------------------------------------------------------------------------
// Persistent step over a batch of D2Q9 members: one block per member, all
// nsteps in the launch with a block barrier between steps.
// -------------------------------------------------------------------------
template <typename T, int NT, int CPT, bool CORR, bool EXT>
__global__ __launch_bounds__(NT) void k_d2q9_members(MemberLaunch a) {
  const MemberDesc d = a.descs[blockIdx.x];
  const int tid = threadIdx.x;
  const uint32_t esz = sizeof(T);
  const uint32_t base = (uint32_t)d.offset;
  int nbad = 0;
  for (int t = 0; t < a.nsteps; ++t) {
    const bool odd = a.pingpong && (t & 1);
    const T* __restrict__ src = (const T*)(odd ? a.bufB : a.bufA);
    T* __restrict__ dst = (T*)(odd ? a.bufA : a.bufB);
    const int64_t sidx = a.step0 + t + 1;
    const bool diag = a.diag_every > 0 && ((sidx % a.diag_every) == 0 || t == a.nsteps - 1);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c0 = 0; c0 < d.ncells; c0 += NT * CPT) {
#pragma unroll
      for (int k = 0; k < CPT; ++k) {
        const int c = c0 + k * NT + tid;
        if (c < d.ncells) {
          const int y = c / d.nx;
          const int x = c - y * d.nx;
          d2q9::C7Fields fm, fp;
          if constexpr (CORR)
            c7_neighbours(src, a.cs, x, y, d.nx, d.ny, d.bcx, d.bcy, base, d.ref, fm, fp);
          uint32_t off[9], self;
          d2q9::pull_offsets(x, y, d.nx, d.ny, d.bcx, d.bcy, base, esz, off, self);
          T f[9], g[9];
#pragma unroll
          for (int q = 0; q < 9; ++q) {
            f[q] = ld(src + (int64_t)q * a.cs, off[q]);
            g[q] = ld(src + (int64_t)(9 + q) * a.cs, off[q]);
          }
          Sums s;
          const bool ok =
              d2q9::collide<T, CORR, EXT>(f, g, d.rt, d.ref, s, &fm, &fp, &d.ext);
          nbad += ok ? 0 : 1;
#pragma unroll
          for (int i = 0; i < 5; ++i) acc[i] += s.v[i];
#pragma unroll
          for (int q = 0; q < 9; ++q) {
            st(dst + (int64_t)q * a.cs, self, f[q]);
            st(dst + (int64_t)(9 + q) * a.cs, self, g[q]);
          }
        }
      }
    }
    if (diag) {
      block_sum5<NT>(acc, tid);
      if (tid == 0)
#pragma unroll
        for (int i = 0; i < 5; ++i) a.partials[(int64_t)blockIdx.x * 5 + i] = acc[i];
    }
    __syncthreads();
  }
  if (nbad) count_bad(a.bad, nbad);
}

// -------------------------------------------------------------------------
// Strip rounds over a batch of members narrow in x and long in y (the
// 4 x 800 tubes of Sec. V.B): every member is cut into segments of whole
// rows, and one block holds a segment's window (owned rows plus halo rows on
// each side, all nx columns) in LDS as [18][NT], one thread per window cell
// (w = row * nx + x). Each launch advances nsteps <= H steps there; halo
// rows absorb the error of the unknown rows beyond the window, which moves
// one row per step (two with the correction term, whose y-neighbour fields
// come from cells one row further out). Per step: pull the 18 values from
// the LDS neighbours (x by the member's rule; y inside the window, wrapped
// only when the window is a whole periodic member, else held at the window
// edge, which is exact at a zero-gradient end), publish the cell's C_7
// fields (CORR), barrier, collide, write back in place, barrier. Cells,
// counts and diagnostics of owned rows only are kept; the arithmetic is that
// of k_d2q9_members, so results are identical bit for bit.
// -------------------------------------------------------------------------
template <typename T, int NT, bool CORR, bool EXT>
__global__ __launch_bounds__(NT) void k_d2q9_strips(TubeRound a) {
  __shared__ T lds[18][NT];
  __shared__ double cf[CORR ? 4 : 1][CORR ? NT : 1];  // x1, gamma, sigma u^2, sigma u
  __shared__ int cok[CORR ? NT : 1];
  const TubeSeg sg = a.segs[blockIdx.x];
  const MemberDesc d = a.descs[sg.member];
  const int nx = d.nx;
  const int w = threadIdx.x;
  const bool live = w < sg.wlen * nx;
  const int r = live ? w / nx : 0;  // window row
  const int x = live ? w - r * nx : 0;
  const bool owned = live && r >= sg.own0 - sg.win0 && r < sg.own1 - sg.win0;
  int y = sg.win0 + r;
  if (y < 0) y += d.ny;
  if (y >= d.ny) y -= d.ny;
  const int64_t gi = d.offset + (int64_t)y * nx + x;
  if (live) {
#pragma unroll
    for (int p = 0; p < 18; ++p) lds[p][w] = ((const T*)a.src)[p * a.cs + gi];
  }
  // window rows of the y - 1 and y + 1 neighbours, columns of x - 1 and x + 1
  int rm = r - 1, rp = r + 1;
  if (rm < 0) rm = sg.left == kEdgeWrap ? sg.wlen - 1 : 0;
  if (rp >= sg.wlen) rp = sg.right == kEdgeWrap ? 0 : sg.wlen - 1;
  const int xm = nbr(x, -1, nx, d.bcx), xp = nbr(x, 1, nx, d.bcx);
  int slot[9];  // pull source of velocity a: the cell at (x, y) - e_a
  slot[0] = r * nx + x;
  slot[1] = r * nx + xm;
  slot[2] = rm * nx + x;
  slot[3] = r * nx + xp;
  slot[4] = rp * nx + x;
  slot[5] = rm * nx + xm;
  slot[6] = rm * nx + xp;
  slot[7] = rp * nx + xp;
  slot[8] = rp * nx + xm;
  if (!live)
#pragma unroll
    for (int q = 0; q < 9; ++q) slot[q] = 0;
  const int sm = rm * nx + x, sp = rp * nx + x;  // C_7 neighbours
  __syncthreads();
  int nbad = 0;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int t = 0; t < a.nsteps; ++t) {
    T f[9], g[9];
    d2q9::Recovered rec;  // with CORR: the recovery behind the published fields
    if (live) {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        f[q] = lds[q][slot[q]];
        g[q] = lds[9 + q][slot[q]];
      }
      if constexpr (CORR) {
        rec = d2q9::recovered<T, EXT>(f, g, d.ref, &d.ext);
        const d2q9::C7Fields F = d2q9::c7_fields(rec.mac, rec.ok);
        cf[0][w] = F.x1;
        cf[1][w] = F.gam;
        cf[2][w] = F.su2;
        cf[3][w] = F.su;
        cok[w] = F.ok ? 1 : 0;
      }
    }
    __syncthreads();
    const int64_t sidx = a.step0 + t + 1;
    const bool diag =
        a.diag_every > 0 && ((sidx % a.diag_every) == 0 || sidx == a.last_step);
    if (live) {
      d2q9::C7Fields fm, fp;
      if constexpr (CORR) {
        fm = d2q9::C7Fields{cf[0][sm], cf[1][sm], cf[2][sm], cf[3][sm], cok[sm] != 0};
        fp = d2q9::C7Fields{cf[0][sp], cf[1][sp], cf[2][sp], cf[3][sp], cok[sp] != 0};
      }
      Sums s;
      bool ok;
      if constexpr (CORR)
        ok = d2q9::collide_recovered<T, true, EXT>(f, g, rec, d.rt, d.ref, s, &fm, &fp, &d.ext);
      else
        ok = d2q9::collide<T, false, EXT>(f, g, d.rt, d.ref, s, nullptr, nullptr, &d.ext);
      if (owned) {
        nbad += ok ? 0 : 1;
        if (diag)
#pragma unroll
          for (int i = 0; i < 5; ++i) acc[i] = s.v[i];
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        lds[q][w] = f[q];
        lds[9 + q][w] = g[q];
      }
    }
    if (diag) {
      if (!owned)
#pragma unroll
        for (int i = 0; i < 5; ++i) acc[i] = 0.0;
      block_sum5<NT>(acc, w);
      if (w == 0)
#pragma unroll
        for (int i = 0; i < 5; ++i) a.partials[(int64_t)blockIdx.x * 5 + i] = acc[i];
    }
    __syncthreads();
  }
  if (owned) {
#pragma unroll
    for (int p = 0; p < 18; ++p) ((T*)a.dst)[p * a.cs + gi] = lds[p][w];
  }
  if (nbad) count_bad(a.bad, nbad);
}

// -------------------------------------------------------------------------
// Tile rounds on one D2Q9 lattice (temporal blocking): a block of NTH threads
// holds the TX x TY window of its tile (the owned cells plus hx / hy halo
// cells a side) in LDS as [18][TX*TY], each thread TX*TY/NTH window cells
// (c = tid + k NTH, i = c mod TX, j = c / TX), and advances nsteps <= H
// steps there before writing the owned cells. Each round reads every window
// cell once and writes every owned cell once, so HBM traffic per cell update
// falls from 2 x 18 values to about (1 + window/owned) x 18 / H. Windows are
// cut at zero-gradient faces (pulls held at the window edge there are exact);
// an axis no longer than the block is one whole window, wrapped if periodic.
// The step itself is that of k_d2q9_strips (pull from LDS, C_7 fields
// published in LDS, collide in registers, write back in place), and gives the
// same results as the one-step kernels bit for bit. Step t + 1 of a round
// updates only the window less t + 1 cells (2(t + 1) rows in y with the
// correction) at each halo edge, which is all the owned cells need, its cells
// dealt to the threads row by row so that whole waves drop out. The owned
// cells are written with plain stores: on 4096^2 lattices (2.4 GB FP32 state)
// that measured 7 % faster per step than nontemporal stores in FP32 and 1 % in
// FP64, as the next round's halo reads of freshly written cells hit in cache.
// -------------------------------------------------------------------------
struct AxisWindow {
  int w0, wlen, own0, own1;  // window start (may be < 0 when periodic), length, owned range
  int left, right;           // edge kinds
};

__device__ __forceinline__ AxisWindow axis_window(int b, int N, int T, int O, int h, int bc) {
  AxisWindow w;
  if (N <= T) {  // the whole axis
    w.w0 = 0;
    w.wlen = N;
    w.own0 = 0;
    w.own1 = N;
    w.left = w.right = bc == 0 ? kEdgeWrap : kEdgeClamp;
    return w;
  }
  w.own0 = b * O;
  w.own1 = min(N, w.own0 + O);
  if (bc == 0) {
    w.w0 = w.own0 - h;
    w.wlen = w.own1 - w.own0 + 2 * h;
    w.left = w.right = kEdgeHalo;
  } else {
    w.w0 = max(0, w.own0 - h);
    const int w1 = min(N, w.own1 + h);
    w.wlen = w1 - w.w0;
    w.left = w.w0 == 0 ? kEdgeClamp : kEdgeHalo;
    w.right = w1 == N ? kEdgeClamp : kEdgeHalo;
  }
  return w;
}

template <typename T, int TX, int TY, int NTH, bool CORR, bool EXT>
__global__ __launch_bounds__(NTH) void k_d2q9_tiles(TileRound a) {
  constexpr int NT = TX * TY;     // window cells
  constexpr int CPT = NT / NTH;   // window cells per thread: c = tid + k * NTH
  static_assert(CPT * NTH == NT, "threads must divide the window");
  constexpr int YS = CORR ? 2 : 1;  // halo rows consumed per step along y
  __shared__ T lds[18][NT];
  __shared__ double cf[CORR ? 4 : 1][CORR ? NT : 1];  // x1, gamma, sigma u^2, sigma u
  __shared__ int cok[CORR ? NT : 1];
  int bx, by, bz;
  block_tile(bx, by, bz);  // the tiles of a row on one XCD: their windows overlap in x
  const AxisWindow X = axis_window(bx, a.nx, TX, a.ox, a.hx, a.bcx);
  const AxisWindow Y = axis_window(by, a.ny, TY, a.oy, a.hy, a.bcy);
  const int tid = threadIdx.x;
  bool owned[CPT];
  int64_t gi[CPT];
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = tid + k * NTH;
    const int i = c % TX, j = c / TX;
    const bool live = i < X.wlen && j < Y.wlen;
    owned[k] = live && X.w0 + i >= X.own0 && X.w0 + i < X.own1 && Y.w0 + j >= Y.own0 &&
               Y.w0 + j < Y.own1;
    int gx = X.w0 + i, gy = Y.w0 + j;
    if (gx < 0) gx += a.nx;
    if (gx >= a.nx) gx -= a.nx;
    if (gy < 0) gy += a.ny;
    if (gy >= a.ny) gy -= a.ny;
    gi[k] = (int64_t)gy * a.nx + gx;
    if (live) {
#pragma unroll
      for (int p = 0; p < 18; ++p) lds[p][c] = ((const T*)a.src)[p * a.cs + gi[k]];
    }
  }
  __syncthreads();
  int nbad = 0;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int t = 0; t < a.nsteps; ++t) {
    // Step s = t + 1 updates the window less s cells (YS s rows) at each halo
    // edge: the owned cells after the round need no more. With the correction
    // the cells one row further out also publish their C_7 fields, which their
    // y-neighbours in the region read. The cells are dealt to the threads row
    // by row (r = tid + k NTH), so whole waves drop out as the region shrinks.
    const int s = t + 1;
    const int i0 = X.left == kEdgeHalo ? s : 0;
    const int i1 = X.wlen - (X.right == kEdgeHalo ? s : 0);
    const int j0 = Y.left == kEdgeHalo ? YS * s : 0;
    const int j1 = Y.wlen - (Y.right == kEdgeHalo ? YS * s : 0);
    const int pj0 = CORR && Y.left == kEdgeHalo ? j0 - 1 : j0;
    const int pj1 = CORR && Y.right == kEdgeHalo ? j1 + 1 : j1;
    const int w = i1 - i0, n = w * (pj1 - pj0);
    // row of slot r: r / w through the hardware FP32 reciprocal (within 1 ulp
    // of 1/w). (r + 1/2) / w lies at least 1/(2w) from an integer; the
    // reciprocal's error and the product's rounding move it by at most 2^-22
    // of itself, under 2^-11 for r < 2^11, which is less than 1/(2w) for
    // w <= 256: the truncation is exact, in 3 instructions per slot where an
    // integer division takes about 25
    static_assert(NT <= 2048 && TX <= 256, "the reciprocal row split needs r < 2^11, w <= 256");
    const float inv_w = __builtin_amdgcn_rcpf((float)w);
    // owned range in window coordinates
    const int oi0 = X.own0 - X.w0, oi1 = X.own1 - X.w0;
    const int oj0 = Y.own0 - Y.w0, oj1 = Y.own1 - Y.w0;
    // every pull of the step lands in registers before the in-place writes
    T f[CPT][9], g[CPT][9];
    d2q9::Recovered rec[CPT];  // with CORR: the recovery behind the published fields
    int cell[CPT], cm[CPT], cp[CPT];
    bool upd[CPT], own[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int r = tid + k * NTH;
      cell[k] = cm[k] = cp[k] = 0;
      upd[k] = own[k] = false;
      if (r < n) {
        const int jr = (int)(((float)r + 0.5f) * inv_w);
        const int i = i0 + (r - jr * w), j = pj0 + jr;
        int im = i - 1, ip = i + 1, jm = j - 1, jp = j + 1;
        if (im < 0) im = X.left == kEdgeWrap ? X.wlen - 1 : 0;
        if (ip >= X.wlen) ip = X.right == kEdgeWrap ? 0 : X.wlen - 1;
        if (jm < 0) jm = Y.left == kEdgeWrap ? Y.wlen - 1 : 0;
        if (jp >= Y.wlen) jp = Y.right == kEdgeWrap ? 0 : Y.wlen - 1;
        // pull source of velocity a: the cell at (i, j) - e_a
        const int sl[9] = {j * TX + i,   j * TX + im,  jm * TX + i,  j * TX + ip, jp * TX + i,
                           jm * TX + im, jm * TX + ip, jp * TX + ip, jp * TX + im};
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          f[k][q] = lds[q][sl[q]];
          g[k][q] = lds[9 + q][sl[q]];
        }
        cell[k] = j * TX + i;
        cm[k] = jm * TX + i;  // C_7 neighbours
        cp[k] = jp * TX + i;
        upd[k] = j >= j0 && j < j1;
        own[k] = i >= oi0 && i < oi1 && j >= oj0 && j < oj1;
        if constexpr (CORR) {
          rec[k] = d2q9::recovered<T, EXT>(f[k], g[k], a.ref, &a.ext);
          const d2q9::C7Fields F = d2q9::c7_fields(rec[k].mac, rec[k].ok);
          cf[0][cell[k]] = F.x1;
          cf[1][cell[k]] = F.gam;
          cf[2][cell[k]] = F.su2;
          cf[3][cell[k]] = F.su;
          cok[cell[k]] = F.ok ? 1 : 0;
        }
      }
    }
    __syncthreads();
    const int64_t sidx = a.step0 + t + 1;
    const bool diag =
        a.diag_every > 0 && ((sidx % a.diag_every) == 0 || sidx == a.last_step);
    if (diag)
#pragma unroll
      for (int q = 0; q < 5; ++q) acc[q] = 0.0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      if (upd[k]) {
        Sums sm5;
        bool ok;
        if constexpr (CORR) {
          const int m = cm[k], p = cp[k];
          const d2q9::C7Fields fm{cf[0][m], cf[1][m], cf[2][m], cf[3][m], cok[m] != 0};
          const d2q9::C7Fields fp{cf[0][p], cf[1][p], cf[2][p], cf[3][p], cok[p] != 0};
          ok = d2q9::collide_recovered<T, true, EXT>(f[k], g[k], rec[k], a.rt, a.ref, sm5, &fm,
                                                     &fp, &a.ext);
        } else {
          ok = d2q9::collide<T, false, EXT>(f[k], g[k], a.rt, a.ref, sm5, nullptr, nullptr,
                                            &a.ext);
        }
        if (own[k]) {
          nbad += ok ? 0 : 1;
          if (diag)
#pragma unroll
            for (int q = 0; q < 5; ++q) acc[q] += sm5.v[q];
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          lds[q][cell[k]] = f[k][q];
          lds[9 + q][cell[k]] = g[k][q];
        }
      }
    }
    if (diag) {
      block_sum5<NTH>(acc, tid);
      if (tid == 0) {
        const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
        for (int q = 0; q < 5; ++q) a.partials[b * 5 + q] = acc[q];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    if (owned[k]) {
      const int c = tid + k * NTH;
      const uint32_t off = (uint32_t)(gi[k] * sizeof(T));
#pragma unroll
      for (int p = 0; p < 18; ++p) st((T*)a.dst + (int64_t)p * a.cs, off, lds[p][c]);
    }
  }
  if (nbad) count_bad(a.bad, nbad);
}

__device__ __forceinline__ int member_of(const MemberDesc* __restrict__ d, int n, int64_t c) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].offset <= c)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <typename T>
__global__ __launch_bounds__(256) void k_d2q9_init(T* state, int64_t cs, const MemberDesc* descs,
                                                   int n_members, const double* n0,
                                                   const double* eps0, const double* u0,
                                                   int64_t ncells) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < ncells;
       i += (int64_t)gridDim.x * 256) {
    const MemberDesc& d = descs[member_of(descs, n_members, i)];
    double f[9], g[9];
    const double P = pressure_of(eps0[i], n0[i], d.ext);
    d2q9::equilibrium_dev(n0[i], eps0[i], P, u0[i], u0[ncells + i], d.ref, f, g);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      state[a * cs + i] = (T)f[a];
      state[(9 + a) * cs + i] = (T)g[a];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_d2q9_export(const T* state, int64_t cs,
                                                     const MemberDesc* descs, int n_members,
                                                     int64_t ncells, double* n, double* eps,
                                                     double* P, double* gamma, double* u,
                                                     double* partials) {
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < ncells;
       i += (int64_t)gridDim.x * 256) {
    const MemberDesc& d = descs[member_of(descs, n_members, i)];
    T f[9], g[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      f[a] = state[a * cs + i];
      g[a] = state[(9 + a) * cs + i];
    }
    double N, E, Mx, My, fs, gs;
    d2q9::cell_sums(f, g, d.ref, N, E, Mx, My, fs, gs);
    acc[0] += N;
    acc[1] += E;
    acc[2] += Mx;
    acc[3] += My;
    Macro m;
    const bool gen = d.ext.general_eos != 0;
    const bool ok = d2q9::recover_model_xy(N, E, Mx, My, d.ext, m);
    const double nan = __builtin_nan("");
    const double e =
        !ok ? nan : (gen ? m.sigma * (1.0 - m.u2) - m.P : 0.75 * m.sigma * (1.0 - m.u2));
    const double gm = ok ? 1.0 / sqrt(1.0 - m.u2) : nan;
    if (n) n[i] = ok ? N / gm : nan;
    if (eps) eps[i] = e;
    if (P) P[i] = !ok ? nan : (gen ? m.P : e / 3.0);
    if (gamma) gamma[i] = gm;
    if (u) {
      u[i] = ok ? m.ux : nan;
      u[ncells + i] = ok ? m.uy : nan;
      u[2 * ncells + i] = ok ? 0.0 : nan;
    }
  }
  block_sum5<256>(acc, threadIdx.x);
  if (threadIdx.x == 0)
    for (int k = 0; k < 5; ++k) partials[(int64_t)blockIdx.x * 5 + k] = acc[k];
}

// Planes [p0, p0 + np) as FP64 populations (reference added back); plane
// p < 9 is f_p, p >= 9 is g_(p-9). out[(p - p0) * ncells + cell].
template <typename T>
__global__ __launch_bounds__(256) void k_d2q9_planes(const T* state, int64_t cs,
                                                     const MemberDesc* descs, int n_members,
                                                     int64_t ncells, int p0, int np,
                                                     double* out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < ncells;
       i += (int64_t)gridDim.x * 256) {
    const Ref ref = descs[member_of(descs, n_members, i)].ref;
    for (int p = p0; p < p0 + np; ++p) {
      const double r = p < 9 ? d2q9::weight(p) * ref.n : d2q9::gref_unit(p - 9) * ref.P;
      out[(int64_t)(p - p0) * ncells + i] = (double)state[p * cs + i] + r;
    }
  }
}

// ------------------------------ variants ---------------------------------
constexpr LatticeVariant kLat2[] = {{64, 1, 1},  {128, 1, 1}, {256, 1, 1}, {64, 4, 1},
                                    {128, 2, 1}, {256, 1, 2}, {256, 1, 4}, {128, 2, 4},
                                    {64, 8, 1},  {128, 4, 1}};
constexpr int kNumLat2 = sizeof(kLat2) / sizeof(kLat2[0]);
// At most 512 threads: the 1024-thread builds spill to scratch (refused by the build).
constexpr MemberVariant kMem2[] = {{256, 1}, {512, 1}, {512, 2}};
constexpr int kNumMem2 = sizeof(kMem2) / sizeof(kMem2[0]);
// strip rounds: threads per block, steps per launch
constexpr TubeVariant kStrip2[] = {{128, 2}, {128, 4}, {256, 4}, {256, 8}, {512, 8}, {512, 16}};
constexpr int kNumStrip2 = sizeof(kStrip2) / sizeof(kStrip2[0]);

int grid2_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

// With the correction term, blocks of one cell per thread and at least 4 rows
// share the neighbours' C_7 fields through LDS (k_d2q9_lattice_c7).
template <int BY, int CY, bool CORR>
constexpr bool kC7Lds = CORR && CY == 1 && BY >= 4;

template <typename T, int BX, int BY, int CY, bool CORR, bool EXT, bool NTS>
void lat2_launch_stores(bool diag, dim3 grid, dim3 block, const void* src, void* dst,
                        const LatticeGeom& g, double* partials, unsigned long long* bad,
                        hipStream_t s) {
  if constexpr (kC7Lds<BY, CY, CORR>) {
    if (diag)
      hipLaunchKernelGGL((k_d2q9_lattice_c7<T, BX, BY, true, EXT, NTS>), grid, block, 0, s,
                         (const T*)src, (T*)dst, g, partials, bad);
    else
      hipLaunchKernelGGL((k_d2q9_lattice_c7<T, BX, BY, false, EXT, NTS>), grid, block, 0, s,
                         (const T*)src, (T*)dst, g, partials, bad);
  } else {
    if (diag)
      hipLaunchKernelGGL((k_d2q9_lattice<T, BX, BY, CY, true, CORR, EXT, NTS>), grid, block, 0,
                         s, (const T*)src, (T*)dst, g, partials, bad);
    else
      hipLaunchKernelGGL((k_d2q9_lattice<T, BX, BY, CY, false, CORR, EXT, NTS>), grid, block, 0,
                         s, (const T*)src, (T*)dst, g, partials, bad);
  }
}

template <typename T, int BX, int BY, int CY, bool CORR, bool EXT>
hipError_t lat2_launch(bool diag, const void* src, void* dst, const LatticeGeom& g,
                       double* partials, unsigned long long* bad, hipStream_t s) {
  dim3 block(BX, BY, 1);
  dim3 grid((g.nx + BX - 1) / BX, (g.ny + BY * CY - 1) / (BY * CY), 1);
  if (g.cached_store)
    lat2_launch_stores<T, BX, BY, CY, CORR, EXT, false>(diag, grid, block, src, dst, g, partials,
                                                        bad, s);
  else
    lat2_launch_stores<T, BX, BY, CY, CORR, EXT, true>(diag, grid, block, src, dst, g, partials,
                                                       bad, s);
  return hipGetLastError();
}

template <typename T, bool CORR, bool EXT>
hipError_t lat2_dispatch(int v, bool diag, const void* src, void* dst, const LatticeGeom& g,
                         double* partials, unsigned long long* bad, hipStream_t s) {
  switch (v) {
    case 0: return lat2_launch<T, 64, 1, 1, CORR, EXT>(diag, src, dst, g, partials, bad, s);
    case 1: return lat2_launch<T, 128, 1, 1, CORR, EXT>(diag, src, dst, g, partials, bad, s);
    case 2: return lat2_launch<T, 256, 1, 1, CORR, EXT>(diag, src, dst, g, partials, bad, s);
    case 3: return lat2_launch<T, 64, 4, 1, CORR, EXT>(diag, src, dst, g, partials, bad, s);
    case 4: return lat2_launch<T, 128, 2, 1, CORR, EXT>(diag, src, dst, g, partials, bad, s);
    case 5: return lat2_launch<T, 256, 1, 2, CORR, EXT>(diag, src, dst, g, partials, bad, s);
    case 6: return lat2_launch<T, 256, 1, 4, CORR, EXT>(diag, src, dst, g, partials, bad, s);
    case 7: return lat2_launch<T, 128, 2, 4, CORR, EXT>(diag, src, dst, g, partials, bad, s);
    case 8: return lat2_launch<T, 64, 8, 1, CORR, EXT>(diag, src, dst, g, partials, bad, s);
    case 9: return lat2_launch<T, 128, 4, 1, CORR, EXT>(diag, src, dst, g, partials, bad, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, bool CORR, bool EXT>
const void* mem2_func(int v) {
  switch (v) {
    case 0: return (const void*)&k_d2q9_members<T, 256, 1, CORR, EXT>;
    case 1: return (const void*)&k_d2q9_members<T, 512, 1, CORR, EXT>;
    case 2: return (const void*)&k_d2q9_members<T, 512, 2, CORR, EXT>;
  }
  return nullptr;
}

// tile rounds: block (= window) shape and steps per launch
constexpr TileVariant kTile2[] = {{32, 16, 2}, {64, 8, 2}, {32, 32, 2}, {64, 16, 2}, {32, 32, 3},
                                  {64, 16, 3}, {32, 16, 3}};
constexpr int kNumTile2 = sizeof(kTile2) / sizeof(kTile2[0]);

// LDS of a tile block: the window's 18 populations, and with the correction
// term its published fields (4 doubles and a flag per cell).
constexpr size_t tile_lds_bytes(size_t esz, int nt, bool corr) {
  return 18 * (size_t)nt * esz + (corr ? (size_t)nt * (4 * sizeof(double) + sizeof(int)) : 0);
}
constexpr size_t kLdsLimit = 160 * 1024;

constexpr int kTileThreads = 512;

template <typename T, int TX, int TY, bool CORR, bool EXT>
hipError_t tile2_launch(const TileRound& a, dim3 grid, hipStream_t s) {
  if constexpr (tile_lds_bytes(sizeof(T), TX * TY, CORR) > kLdsLimit) {
    return hipErrorInvalidValue;  // refused on the host (d2q9_tile_fits)
  } else {
    hipLaunchKernelGGL((k_d2q9_tiles<T, TX, TY, kTileThreads, CORR, EXT>), grid,
                       dim3(kTileThreads, 1, 1), 0, s, a);
    return hipGetLastError();
  }
}

template <typename T, bool CORR, bool EXT>
hipError_t tile2_dispatch(int v, const TileRound& a, dim3 grid, hipStream_t s) {
  switch (v) {
    case 0: return tile2_launch<T, 32, 16, CORR, EXT>(a, grid, s);
    case 1: return tile2_launch<T, 64, 8, CORR, EXT>(a, grid, s);
    case 2: return tile2_launch<T, 32, 32, CORR, EXT>(a, grid, s);
    case 3: return tile2_launch<T, 64, 16, CORR, EXT>(a, grid, s);
    case 4: return tile2_launch<T, 32, 32, CORR, EXT>(a, grid, s);
    case 5: return tile2_launch<T, 64, 16, CORR, EXT>(a, grid, s);
    case 6: return tile2_launch<T, 32, 16, CORR, EXT>(a, grid, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, bool CORR, bool EXT>
const void* strip2_func(int v) {
  switch (v) {
    case 0: return (const void*)&k_d2q9_strips<T, 128, CORR, EXT>;
    case 1: return (const void*)&k_d2q9_strips<T, 128, CORR, EXT>;
    case 2: return (const void*)&k_d2q9_strips<T, 256, CORR, EXT>;
    case 3: return (const void*)&k_d2q9_strips<T, 256, CORR, EXT>;
    case 4: return (const void*)&k_d2q9_strips<T, 512, CORR, EXT>;
    case 5: return (const void*)&k_d2q9_strips<T, 512, CORR, EXT>;
  }
  return nullptr;
}

}  // namespace

int d2q9_num_lattice_variants() { return kNumLat2; }

int d2q9_lattice_partials(int v, const LatticeGeom& g) {
  const LatticeVariant lv = kLat2[v];
  return ((g.nx + lv.bx - 1) / lv.bx) * ((g.ny + lv.by * lv.cz - 1) / (lv.by * lv.cz));
}

const char* d2q9_lattice_kernel_name(int precision, int v) {
  static const char* n32[] = {"k_d2q9_lattice<float,64,1,1>",  "k_d2q9_lattice<float,128,1,1>",
                              "k_d2q9_lattice<float,256,1,1>", "k_d2q9_lattice<float,64,4,1>",
                              "k_d2q9_lattice<float,128,2,1>", "k_d2q9_lattice<float,256,1,2>",
                              "k_d2q9_lattice<float,256,1,4>", "k_d2q9_lattice<float,128,2,4>",
                              "k_d2q9_lattice<float,64,8,1>",  "k_d2q9_lattice<float,128,4,1>"};
  static const char* n64[] = {
      "k_d2q9_lattice<double,64,1,1>",  "k_d2q9_lattice<double,128,1,1>",
      "k_d2q9_lattice<double,256,1,1>", "k_d2q9_lattice<double,64,4,1>",
      "k_d2q9_lattice<double,128,2,1>", "k_d2q9_lattice<double,256,1,2>",
      "k_d2q9_lattice<double,256,1,4>", "k_d2q9_lattice<double,128,2,4>",
      "k_d2q9_lattice<double,64,8,1>",  "k_d2q9_lattice<double,128,4,1>"};
  static_assert(sizeof(n32) / sizeof(n32[0]) == kNumLat2, "one name per variant");
  static_assert(sizeof(n64) / sizeof(n64[0]) == kNumLat2, "one name per variant");
  if (v < 0 || v >= kNumLat2) return "?";
  return precision ? n32[v] : n64[v];
}

template <typename T>
hipError_t lat2_modes(int v, bool diag, bool corr, bool ext, const void* src, void* dst,
                      const LatticeGeom& g, double* partials, unsigned long long* bad,
                      hipStream_t s) {
  if (corr)
    return ext ? lat2_dispatch<T, true, true>(v, diag, src, dst, g, partials, bad, s)
              : lat2_dispatch<T, true, false>(v, diag, src, dst, g, partials, bad, s);
  return ext ? lat2_dispatch<T, false, true>(v, diag, src, dst, g, partials, bad, s)
            : lat2_dispatch<T, false, false>(v, diag, src, dst, g, partials, bad, s);
}

hipError_t d2q9_launch_step_lattice(int precision, int v, bool diag, bool corr, bool ext,
                                    const void* src, void* dst, const LatticeGeom& g,
                                    double* partials, unsigned long long* bad, hipStream_t s) {
  if (precision) return lat2_modes<float>(v, diag, corr, ext, src, dst, g, partials, bad, s);
  return lat2_modes<double>(v, diag, corr, ext, src, dst, g, partials, bad, s);
}

int d2q9_num_member_variants() { return kNumMem2; }

template <typename T>
const void* mem2_modes(int v, bool corr, bool ext) {
  if (corr) return ext ? mem2_func<T, true, true>(v) : mem2_func<T, true, false>(v);
  return ext ? mem2_func<T, false, true>(v) : mem2_func<T, false, false>(v);
}

hipError_t d2q9_member_kernel(int precision, int v, bool corr, bool ext, const void** func,
                              dim3* block) {
  if (v < 0 || v >= kNumMem2) return hipErrorInvalidValue;
  *func = precision ? mem2_modes<float>(v, corr, ext) : mem2_modes<double>(v, corr, ext);
  *block = dim3(kMem2[v].nt, 1, 1);
  return hipSuccess;
}

const char* d2q9_member_kernel_name(int precision, int v) {
  static const char* n32[] = {"k_d2q9_members<float,256,1>", "k_d2q9_members<float,512,1>",
                              "k_d2q9_members<float,512,2>"};
  static const char* n64[] = {"k_d2q9_members<double,256,1>", "k_d2q9_members<double,512,1>",
                              "k_d2q9_members<double,512,2>"};
  if (v < 0 || v >= kNumMem2) return "?";
  return precision ? n32[v] : n64[v];
}

int d2q9_num_tile_variants() { return kNumTile2; }
bool d2q9_tile_fits(int precision, int v, bool corr) {
  return tile_lds_bytes(precision ? 4 : 8, kTile2[v].tx * kTile2[v].ty, corr) <= kLdsLimit;
}
TileVariant d2q9_tile_variant(int i) { return kTile2[i]; }

template <typename T>
hipError_t tile2_modes(int v, bool corr, bool ext, const TileRound& a, dim3 grid, hipStream_t s) {
  if (corr)
    return ext ? tile2_dispatch<T, true, true>(v, a, grid, s)
               : tile2_dispatch<T, true, false>(v, a, grid, s);
  return ext ? tile2_dispatch<T, false, true>(v, a, grid, s)
             : tile2_dispatch<T, false, false>(v, a, grid, s);
}

hipError_t d2q9_launch_tiles(int precision, int v, bool corr, bool ext, const TileRound& a,
                             dim3 grid, hipStream_t s) {
  if (v < 0 || v >= kNumTile2) return hipErrorInvalidValue;
  return precision ? tile2_modes<float>(v, corr, ext, a, grid, s)
                   : tile2_modes<double>(v, corr, ext, a, grid, s);
}

const char* d2q9_tile_kernel_name(int precision, int v) {
  static const char* n32[] = {"k_d2q9_tiles<float,32,16>/h2", "k_d2q9_tiles<float,64,8>/h2",
                              "k_d2q9_tiles<float,32,32>/h2", "k_d2q9_tiles<float,64,16>/h2",
                              "k_d2q9_tiles<float,32,32>/h3", "k_d2q9_tiles<float,64,16>/h3",
                              "k_d2q9_tiles<float,32,16>/h3"};
  static const char* n64[] = {"k_d2q9_tiles<double,32,16>/h2", "k_d2q9_tiles<double,64,8>/h2",
                              "k_d2q9_tiles<double,32,32>/h2", "k_d2q9_tiles<double,64,16>/h2",
                              "k_d2q9_tiles<double,32,32>/h3", "k_d2q9_tiles<double,64,16>/h3",
                              "k_d2q9_tiles<double,32,16>/h3"};
  static_assert(sizeof(n32) / sizeof(n32[0]) == kNumTile2, "one name per variant");
  static_assert(sizeof(n64) / sizeof(n64[0]) == kNumTile2, "one name per variant");
  if (v < 0 || v >= kNumTile2) return "?";
  return precision ? n32[v] : n64[v];
}

int d2q9_num_strip_variants() { return kNumStrip2; }
TubeVariant d2q9_strip_variant(int i) { return kStrip2[i]; }

template <typename T>
const void* strip2_modes(int v, bool corr, bool ext) {
  if (corr) return ext ? strip2_func<T, true, true>(v) : strip2_func<T, true, false>(v);
  return ext ? strip2_func<T, false, true>(v) : strip2_func<T, false, false>(v);
}

hipError_t d2q9_strip_kernel(int precision, int v, bool corr, bool ext, const void** func,
                             dim3* block) {
  if (v < 0 || v >= kNumStrip2) return hipErrorInvalidValue;
  *func = precision ? strip2_modes<float>(v, corr, ext) : strip2_modes<double>(v, corr, ext);
  *block = dim3(kStrip2[v].nt, 1, 1);
  return hipSuccess;
}

const char* d2q9_strip_kernel_name(int precision, int v) {
  static const char* n32[] = {"k_d2q9_strips<float,128>/h2", "k_d2q9_strips<float,128>/h4",
                              "k_d2q9_strips<float,256>/h4", "k_d2q9_strips<float,256>/h8",
                              "k_d2q9_strips<float,512>/h8", "k_d2q9_strips<float,512>/h16"};
  static const char* n64[] = {"k_d2q9_strips<double,128>/h2", "k_d2q9_strips<double,128>/h4",
                              "k_d2q9_strips<double,256>/h4", "k_d2q9_strips<double,256>/h8",
                              "k_d2q9_strips<double,512>/h8", "k_d2q9_strips<double,512>/h16"};
  if (v < 0 || v >= kNumStrip2) return "?";
  return precision ? n32[v] : n64[v];
}

hipError_t d2q9_launch_init(int precision, void* state, int64_t cs, const MemberDesc* descs,
                            int n_members, const double* n0, const double* eps0,
                            const double* u0, int64_t ncells, hipStream_t s) {
  dim3 grid(grid2_for(ncells));
  if (precision)
    hipLaunchKernelGGL(k_d2q9_init<float>, grid, dim3(256), 0, s, (float*)state, cs, descs,
                       n_members, n0, eps0, u0, ncells);
  else
    hipLaunchKernelGGL(k_d2q9_init<double>, grid, dim3(256), 0, s, (double*)state, cs, descs,
                       n_members, n0, eps0, u0, ncells);
  return hipGetLastError();
}

hipError_t d2q9_launch_export(int precision, const void* state, int64_t cs,
                              const MemberDesc* descs, int n_members, int64_t ncells, double* n,
                              double* eps, double* P, double* gamma, double* u,
                              double* partials, int nparts, hipStream_t s) {
  if (precision)
    hipLaunchKernelGGL(k_d2q9_export<float>, dim3(nparts), dim3(256), 0, s, (const float*)state,
                       cs, descs, n_members, ncells, n, eps, P, gamma, u, partials);
  else
    hipLaunchKernelGGL(k_d2q9_export<double>, dim3(nparts), dim3(256), 0, s,
                       (const double*)state, cs, descs, n_members, ncells, n, eps, P, gamma, u,
                       partials);
  return hipGetLastError();
}

hipError_t d2q9_launch_population_planes(int precision, const void* state, int64_t cs,
                                         const MemberDesc* descs, int n_members, int64_t ncells,
                                         int p0, int np, double* out, hipStream_t s) {
  dim3 grid(grid2_for(ncells));
  if (precision)
    hipLaunchKernelGGL(k_d2q9_planes<float>, grid, dim3(256), 0, s, (const float*)state, cs,
                       descs, n_members, ncells, p0, np, out);
  else
    hipLaunchKernelGGL(k_d2q9_planes<double>, grid, dim3(256), 0, s, (const double*)state, cs,
                       descs, n_members, ncells, p0, np, out);
  return hipGetLastError();
}

}  // namespace rlb
