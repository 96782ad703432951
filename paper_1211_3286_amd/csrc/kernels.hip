// Kernels of the relativistic MRT lattice Boltzmann step for gfx950.
//
// Population storage (one buffer): 38 planes of cs elements, planes 0..18 hold
// f_a and planes 19..37 hold g_a (velocity order of rlb.h); a cell's element
// in every plane sits at the same index. Two such buffers alternate (A/B):
// a step pulls from one and writes the other, so it is race-free.
//
// The fused step kernel reads 38 values per cell (streaming with periodic or
// zero-gradient sources), collides in registers (cell.hpp) and writes 38
// values: 2 x 38 x sizeof(T) bytes of HBM traffic per cell update, no reuse.
// Loads use a uniform plane base plus a 32-bit byte offset per lane; stores
// are nontemporal (written once, read by the next step from HBM).

#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "internal.hpp"

namespace rlb {

namespace {

// -------------------------------------------------------------------------
// Fused step on one lattice: grid (ceil(nx/BX), ceil(ny/BY), ceil(nz/CZ)),
// block (BX, BY); each thread updates CZ cells along z. EXT: relaxation times
// of each cell from eta/s. Tiles are taken in the row-per-XCD order of
// block_tile. NTS: nontemporal stores; without, plain stores, which the host
// picks when the double-buffered state fits the memory-side cache, so that the
// next step reads it back from there. (The store kind is a template argument:
// two store loops that differ only in the hint behind a run-time branch get
// merged by the compiler, which keeps the plain form.)
// -------------------------------------------------------------------------
template <typename T, int BX, int BY, int CZ, bool DIAG, bool EXT, bool NTS>
__global__ __launch_bounds__(BX* BY) void k_step_lattice(const T* __restrict__ src,
                                                        T* __restrict__ dst, LatticeGeom geo,
                                                        double* __restrict__ partials,
                                                        unsigned long long* __restrict__ bad) {
  int bx, by, bz;
  block_tile(bx, by, bz);
  const int x = bx * BX + threadIdx.x;
  const int y = by * BY + threadIdx.y;
  const int tid = threadIdx.y * BX + threadIdx.x;
  const bool act = (x < geo.nx) && (y < geo.ny);
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int nbad = 0;
  const uint32_t esz = sizeof(T);
#pragma unroll 1
  for (int k = 0; k < CZ; ++k) {
    const int z = bz * CZ + k;
    if (act && z < geo.nz) {
      uint32_t off[19], self;
      pull_offsets(x, y, z, geo.nx, geo.ny, geo.nz, geo.bcx, geo.bcy, geo.bcz, 0u, esz, off,
                   self);
      if constexpr (!EXT && (sizeof(T) == 8 || CZ == 1)) {
        // g first (its recovery needs no f), then f with the recovered
        // velocity: one distribution's 19 values in flight at a time. FP64:
        // 142 instead of 154 VGPRs, 1.5 % faster; FP32 with one cell per
        // thread: 0.3-0.5 % faster (with several cells per thread FP32 lost
        // 2-9 %, and loads both at once). The arithmetic is that of collide(),
        // bit for bit. (The relaxation times from eta/s and the general
        // equation of state need N before the recovery, so the EXT kernels
        // load both at once.)
        T g[19];
#pragma unroll
        for (int a = 0; a < 19; ++a) g[a] = ld(src + (int64_t)(19 + a) * geo.cs, off[a]);
        double E, Mx, My, Mz, gs;
        g_sums(g, geo.ref, E, Mx, My, Mz, gs);
        Macro mac;
        const bool ok = recover(E, Mx, My, Mz, mac);
        if (ok) collide_g(g, Mx, My, Mz, gs, mac, geo.rt, geo.ref);
#pragma unroll
        for (int a = 0; a < 19; ++a) {
          if constexpr (NTS)
            st_nt(dst + (int64_t)(19 + a) * geo.cs, self, g[a]);
          else
            st(dst + (int64_t)(19 + a) * geo.cs, self, g[a]);
        }
        T f[19];
#pragma unroll
        for (int a = 0; a < 19; ++a) f[a] = ld(src + (int64_t)a * geo.cs, off[a]);
        double fs = 0.0;
#pragma unroll
        for (int a = 0; a < 19; ++a) fs += (double)f[a];
        const double N = geo.ref.n + fs;
        if (ok) collide_f(f, N, fs, mac, geo.rt, geo.ref);
#pragma unroll
        for (int a = 0; a < 19; ++a) {
          if constexpr (NTS)
            st_nt(dst + (int64_t)a * geo.cs, self, f[a]);
          else
            st(dst + (int64_t)a * geo.cs, self, f[a]);
        }
        nbad += ok ? 0 : 1;
        if (DIAG) {
          acc[0] += N;
          acc[1] += E;
          acc[2] += Mx;
          acc[3] += My;
          acc[4] += Mz;
        }
      } else {
        T f[19], g[19];
#pragma unroll
        for (int a = 0; a < 19; ++a) {
          f[a] = ld(src + (int64_t)a * geo.cs, off[a]);
          g[a] = ld(src + (int64_t)(19 + a) * geo.cs, off[a]);
        }
        Sums s;
        const bool ok = collide<T, EXT>(f, g, geo.rt, geo.ref, s, &geo.ext);
        nbad += ok ? 0 : 1;
        if (DIAG)
#pragma unroll
          for (int i = 0; i < 5; ++i) acc[i] += s.v[i];
#pragma unroll
        for (int a = 0; a < 19; ++a) {
          if constexpr (NTS) {
            st_nt(dst + (int64_t)a * geo.cs, self, f[a]);
            st_nt(dst + (int64_t)(19 + a) * geo.cs, self, g[a]);
          } else {
            st(dst + (int64_t)a * geo.cs, self, f[a]);
            st(dst + (int64_t)(19 + a) * geo.cs, self, g[a]);
          }
        }
      }
    }
  }
  if (nbad) count_bad(bad, nbad);
  if (DIAG) {
    block_sum5<BX * BY>(acc, tid);
    if (tid == 0) {
      const int64_t b = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
#pragma unroll
      for (int i = 0; i < 5; ++i) partials[b * 5 + i] = acc[i];
    }
  }
}

// -------------------------------------------------------------------------
// Persistent step over a batch: one block per member, all nsteps inside the
// launch with a block barrier between steps (members are independent, so no
// grid-wide synchronisation exists). Each thread updates CPT cells per sweep,
// interleaved by NT so every load instruction is coalesced.
// -------------------------------------------------------------------------
template <typename T, int NT, int CPT, bool EXT>
__global__ __launch_bounds__(NT) void k_step_members(MemberLaunch a) {
  const MemberDesc d = a.descs[blockIdx.x];
  const int tid = threadIdx.x;
  const uint32_t esz = sizeof(T);
  const uint32_t base = (uint32_t)d.offset;
  const bool tube = d.nx == 1 && d.ny == 1;
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
          int x = 0, y = 0, z = c;  // quasi-1D member (1 x 1 x L): no division
          if (!tube) {
            x = c % d.nx;
            const int yz = c / d.nx;
            y = yz % d.ny;
            z = yz / d.ny;
          }
          uint32_t off[19], self;
          pull_offsets(x, y, z, d.nx, d.ny, d.nz, d.bcx, d.bcy, d.bcz, base, esz, off, self);
          T f[19], g[19];
#pragma unroll
          for (int q = 0; q < 19; ++q) {
            f[q] = ld(src + (int64_t)q * a.cs, off[q]);
            g[q] = ld(src + (int64_t)(19 + q) * a.cs, off[q]);
          }
          Sums s;
          const bool ok = collide<T, EXT>(f, g, d.rt, d.ref, s, &d.ext);
          nbad += ok ? 0 : 1;
#pragma unroll
          for (int i = 0; i < 5; ++i) acc[i] += s.v[i];
#pragma unroll
          for (int q = 0; q < 19; ++q) {
            st(dst + (int64_t)q * a.cs, self, f[q]);
            st(dst + (int64_t)(19 + q) * a.cs, self, g[q]);
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
// Segmented persistent step over a batch: one block per segment (a range of
// whole z-planes of one member), all nsteps inside the launch. Before step t
// a segment waits until its two neighbour segments have completed t steps
// (their planes z0-1 and z1 are pulled, and they read this segment's planes
// of the buffer it is about to overwrite). After its step every thread
// makes its stores visible device-wide before thread 0 publishes the flag
// with release semantics. A wait that exceeds spin_limit polls sets *error
// and ends the launch for that block (every block reaches the exit).
// -------------------------------------------------------------------------
__device__ __forceinline__ bool wait_flag(const unsigned long long* f, unsigned long long target,
                                          int spin_limit) {
  for (int i = 0; i < spin_limit; ++i) {
    if (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= target) return true;
    __builtin_amdgcn_s_sleep(2);
  }
  return false;
}

template <typename T, int NT, int CPT>
__global__ __launch_bounds__(NT) void k_step_segments(SegLaunch a) {
  const Segment sg = a.segs[blockIdx.x];
  const MemberDesc d = a.descs[sg.member];
  const int tid = threadIdx.x;
  const uint32_t esz = sizeof(T);
  const uint32_t base = (uint32_t)d.offset;
  const int plane = d.nx * d.ny;
  const bool tube = plane == 1;
  const int c_begin = sg.z0 * plane, c_end = sg.z1 * plane;
  __shared__ int s_abort;
  int nbad = 0;
  for (int t = 0; t < a.nsteps; ++t) {
    const unsigned long long target = a.epoch + (unsigned long long)t;
    if (tid == 0) {
      bool ok = true;
      if (sg.left >= 0) ok = wait_flag(a.flags + sg.left, target, a.spin_limit);
      if (ok && sg.right >= 0) ok = wait_flag(a.flags + sg.right, target, a.spin_limit);
      s_abort = ok ? 0 : 1;
      if (!ok) atomicOr(a.error, 1);
    }
    __syncthreads();
    if (s_abort) break;
    const bool odd = a.pingpong && (t & 1);
    const T* __restrict__ src = (const T*)(odd ? a.bufB : a.bufA);
    T* __restrict__ dst = (T*)(odd ? a.bufA : a.bufB);
    const int64_t sidx = a.step0 + t + 1;
    const bool diag = a.diag_every > 0 && ((sidx % a.diag_every) == 0 || t == a.nsteps - 1);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c0 = c_begin; c0 < c_end; c0 += NT * CPT) {
#pragma unroll
      for (int k = 0; k < CPT; ++k) {
        const int c = c0 + k * NT + tid;
        if (c < c_end) {
          int x = 0, y = 0, z = c;  // quasi-1D member (1 x 1 x L): no division
          if (!tube) {
            x = c % d.nx;
            const int yz = c / d.nx;
            y = yz % d.ny;
            z = yz / d.ny;
          }
          uint32_t off[19], self;
          pull_offsets(x, y, z, d.nx, d.ny, d.nz, d.bcx, d.bcy, d.bcz, base, esz, off, self);
          T f[19], g[19];
#pragma unroll
          for (int q = 0; q < 19; ++q) {
            f[q] = ld(src + (int64_t)q * a.cs, off[q]);
            g[q] = ld(src + (int64_t)(19 + q) * a.cs, off[q]);
          }
          Sums s;
          const bool ok = collide<T>(f, g, d.rt, d.ref, s);
          nbad += ok ? 0 : 1;
#pragma unroll
          for (int i = 0; i < 5; ++i) acc[i] += s.v[i];
#pragma unroll
          for (int q = 0; q < 19; ++q) {
            st(dst + (int64_t)q * a.cs, self, f[q]);
            st(dst + (int64_t)(19 + q) * a.cs, self, g[q]);
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
    __threadfence();
    __syncthreads();
    if (tid == 0)
      __hip_atomic_store(a.flags + blockIdx.x, target + 1ull, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
  if (nbad) count_bad(a.bad, nbad);
}

// -------------------------------------------------------------------------
// Tube rounds: one block per TubeSeg, one thread per window cell, all
// populations of the window in LDS as [38][NT] (consecutive threads touch
// consecutive words). Per step: every thread pulls its 38 values from the
// LDS neighbours (a 1 x 1 x L lattice streams only along z: the x and y
// components of e wrap onto the same cell), barrier, collides in registers,
// writes them back to its own slot, barrier. Inadmissible counts and
// diagnostics cover owned cells only (halo cells are computed twice). EXT:
// relaxation times from eta/s and the general equation of state, per cell.
// -------------------------------------------------------------------------
template <typename T, int NT, bool EXT>
__global__ __launch_bounds__(NT) void k_step_tubes(TubeRound a) {
  __shared__ T lds[38][NT];
  const TubeSeg sg = a.segs[blockIdx.x];
  const MemberDesc d = a.descs[sg.member];
  const int w = threadIdx.x;
  const int L = d.nz;
  const bool live = w < sg.wlen;
  const int own_lo = sg.own0 - sg.win0, own_hi = sg.own1 - sg.win0;
  const bool owned = w >= own_lo && w < own_hi;
  // global cell of window cell w
  int z = sg.win0 + w;
  if (z < 0) z += L;
  if (z >= L) z -= L;
  const int64_t gi = d.offset + z;
  if (live) {
#pragma unroll
    for (int p = 0; p < 38; ++p) lds[p][w] = ((const T*)a.src)[p * a.cs + gi];
  }
  // pull sources inside the window for e_z = +1 (from w-1) and e_z = -1 (from w+1)
  int sp = w - 1, sm = w + 1;
  if (sp < 0) sp = sg.left == kEdgeWrap ? sg.wlen - 1 : 0;
  if (sm >= sg.wlen) sm = sg.right == kEdgeWrap ? 0 : sg.wlen - 1;
  if (!live) sp = sm = 0;
  __syncthreads();
  int nbad = 0;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int t = 0; t < a.nsteps; ++t) {
    T f[19], g[19];
    if (live) {
#pragma unroll
      for (int q = 0; q < 19; ++q) {
        const int src = ez(q) > 0 ? sp : (ez(q) < 0 ? sm : w);
        f[q] = lds[q][src];
        g[q] = lds[19 + q][src];
      }
    }
    __syncthreads();
    const int64_t sidx = a.step0 + t + 1;
    const bool diag =
        a.diag_every > 0 && ((sidx % a.diag_every) == 0 || sidx == a.last_step);
    if (live) {
      Sums s;
      const bool ok = collide<T, EXT>(f, g, d.rt, d.ref, s, &d.ext);
      if (owned) {
        nbad += ok ? 0 : 1;
        if (diag)
#pragma unroll
          for (int i = 0; i < 5; ++i) acc[i] = s.v[i];
      }
#pragma unroll
      for (int q = 0; q < 19; ++q) {
        lds[q][w] = f[q];
        lds[19 + q][w] = g[q];
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
    for (int p = 0; p < 38; ++p) ((T*)a.dst)[p * a.cs + gi] = lds[p][w];
  }
  if (nbad) count_bad(a.bad, nbad);
}

__device__ __forceinline__ int find_member(const MemberDesc* __restrict__ d, int n, int64_t c) {
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

// Mean n gamma and eps/3 of each member's initial fields (its reference
// state), in two deterministic passes: kRefBlocks partial sums per member,
// then one block per member adds them in order.
__global__ __launch_bounds__(256) void k_member_ref_parts(const MemberDesc* descs,
                                                          const double* n0, const double* eps0,
                                                          const double* u0, int64_t ncells,
                                                          double* parts) {
  const MemberDesc& d = descs[blockIdx.y];
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int c = blockIdx.x * 256 + threadIdx.x; c < d.ncells; c += kRefBlocks * 256) {
    const int64_t i = d.offset + c;
    const double ux = u0[i], uy = u0[ncells + i], uz = u0[2 * ncells + i];
    v[0] += n0[i] / sqrt(1.0 - (ux * ux + uy * uy + uz * uz));
    v[1] += eps0[i];
  }
  block_sum5<256>(v, threadIdx.x);
  if (threadIdx.x == 0) {
    const int64_t b = (int64_t)blockIdx.y * kRefBlocks + blockIdx.x;
    for (int k = 0; k < 5; ++k) parts[b * 5 + k] = v[k];
  }
}

__global__ __launch_bounds__(64) void k_member_ref_final(MemberDesc* descs, const double* parts) {
  if (threadIdx.x != 0) return;
  MemberDesc& d = descs[blockIdx.x];
  double sn = 0.0, se = 0.0;
  for (int b = 0; b < kRefBlocks; ++b) {
    sn += parts[((int64_t)blockIdx.x * kRefBlocks + b) * 5 + 0];
    se += parts[((int64_t)blockIdx.x * kRefBlocks + b) * 5 + 1];
  }
  d.ref.n = sn / d.ncells;
  d.ref.P = se / (3.0 * d.ncells);
}

__global__ __launch_bounds__(256) void k_validate(const double* n0, const double* eps0,
                                                  const double* u0, int64_t ncells, int planar,
                                                  const MemberDesc* descs, int n_members,
                                                  unsigned long long* count) {
  int nb = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < ncells;
       i += (int64_t)gridDim.x * 256) {
    const double ux = u0[i], uy = u0[ncells + i], uz = u0[2 * ncells + i];
    const double uu = ux * ux + uy * uy + uz * uz;
    const Ext& x = descs[find_member(descs, n_members, i)].ext;
    const bool ok = (eps0[i] > 0.0) && (n0[i] >= 0.0) && (uu < 1.0) && (n0[i] < INFINITY) &&
                    (eps0[i] < INFINITY) && (!planar || uz == 0.0) &&
                    (!x.general_eos || eps0[i] - x.mass * n0[i] > 0.0);
    nb += ok ? 0 : 1;
  }
  if (nb) atomicAdd(count, (unsigned long long)nb);
}

template <typename T>
__global__ __launch_bounds__(256) void k_init(T* state, int64_t cs, const MemberDesc* descs,
                                              int n_members, const double* n0,
                                              const double* eps0, const double* u0,
                                              int64_t ncells) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < ncells;
       i += (int64_t)gridDim.x * 256) {
    const MemberDesc& d = descs[find_member(descs, n_members, i)];
    double f[19], g[19];
    const double P = pressure_of(eps0[i], n0[i], d.ext);
    equilibrium_dev(n0[i], eps0[i], P, u0[i], u0[ncells + i], u0[2 * ncells + i], d.ref, f, g);
#pragma unroll
    for (int a = 0; a < 19; ++a) {
      state[a * cs + i] = (T)f[a];
      state[(19 + a) * cs + i] = (T)g[a];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_export(const T* state, int64_t cs,
                                                const MemberDesc* descs, int n_members,
                                                int64_t ncells, double* n, double* eps,
                                                double* P, double* gamma, double* u,
                                                double* partials) {
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < ncells;
       i += (int64_t)gridDim.x * 256) {
    const MemberDesc& d = descs[find_member(descs, n_members, i)];
    T f[19], g[19];
#pragma unroll
    for (int a = 0; a < 19; ++a) {
      f[a] = state[a * cs + i];
      g[a] = state[(19 + a) * cs + i];
    }
    double N, E, Mx, My, Mz, fs, gs;
    cell_sums(f, g, d.ref, N, E, Mx, My, Mz, fs, gs);
    acc[0] += N;
    acc[1] += E;
    acc[2] += Mx;
    acc[3] += My;
    acc[4] += Mz;
    Macro m;
    const bool gen = d.ext.general_eos != 0;
    const bool ok = recover_model(N, E, Mx, My, Mz, d.ext, m);
    const double nan = __builtin_nan("");
    // eps = (eps + P) - P; for P = eps/3 the closed form 3/4 sigma (1 - u^2)
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
      u[2 * ncells + i] = ok ? m.uz : nan;
    }
  }
  block_sum5<256>(acc, threadIdx.x);
  if (threadIdx.x == 0)
    for (int k = 0; k < 5; ++k) partials[(int64_t)blockIdx.x * 5 + k] = acc[k];
}

// Planes [p0, p0 + np) of the state as FP64 populations (reference added back);
// plane p < 19 is f_p, plane p >= 19 is g_(p-19). out[(p - p0) * ncells + cell].
template <typename T>
__global__ __launch_bounds__(256) void k_population_planes(const T* state, int64_t cs,
                                                           const MemberDesc* descs, int n_members,
                                                           int64_t ncells, int p0, int np,
                                                           double* out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < ncells;
       i += (int64_t)gridDim.x * 256) {
    const Ref ref = descs[find_member(descs, n_members, i)].ref;
    for (int p = p0; p < p0 + np; ++p) {
      const double r = p < 19 ? weight(p) * ref.n : gref_unit(p - 19) * ref.P;
      out[(int64_t)(p - p0) * ncells + i] = (double)state[p * cs + i] + r;
    }
  }
}

// Deterministic sum of nparts partial 5-vectors (single block).
__global__ __launch_bounds__(256) void k_reduce(const double* partials, int nparts, double* out) {
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < nparts; j += 256)
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] += partials[(int64_t)j * 5 + k];
  block_sum5<256>(v, threadIdx.x);
  if (threadIdx.x == 0)
    for (int k = 0; k < 5; ++k) out[k] = v[k];
}

// ------------------------------ variants ---------------------------------
// The /w3 forms reserve 44 KiB of LDS per 256-thread block that the kernel
// never touches: 3 blocks fit in a CU's 160 KiB where 4 would by registers, so
// they run 3 waves per SIMD instead of 4. On 512^3 FP32 lattices the 256 x 1
// block ran 2 % faster so (fewer streams in flight per channel); on 256^3
// the blocks were within 1 %.
constexpr unsigned kOcc3Lds = 44 * 1024;
constexpr LatticeVariant kLat[] = {{64, 1, 1},  {64, 4, 1},  {128, 2, 1}, {256, 1, 1},
                                   {64, 4, 2},  {256, 1, 2}, {128, 2, 4}, {256, 1, 4},
                                   {128, 2, 1}, {256, 1, 1}};
constexpr int kNumLat = sizeof(kLat) / sizeof(kLat[0]);
// At most 512 threads: with 1024 (4 waves per SIMD, at most 128 VGPRs) every
// member build spills to scratch, which the build refuses for every kernel.
constexpr MemberVariant kMem[] = {{256, 1}, {512, 1}, {256, 2}, {512, 2}};
constexpr int kNumMem = sizeof(kMem) / sizeof(kMem[0]);

constexpr MemberVariant kSeg[] = {{256, 1}, {256, 2}, {512, 1}, {128, 4}, {256, 4}};
constexpr int kNumSeg = sizeof(kSeg) / sizeof(kSeg[0]);

template <typename T>
const void* seg_func(int v) {
  switch (v) {
    case 0: return (const void*)&k_step_segments<T, 256, 1>;
    case 1: return (const void*)&k_step_segments<T, 256, 2>;
    case 2: return (const void*)&k_step_segments<T, 512, 1>;
    case 3: return (const void*)&k_step_segments<T, 128, 4>;
    case 4: return (const void*)&k_step_segments<T, 256, 4>;
  }
  return nullptr;
}

constexpr TubeVariant kTube[] = {{256, 8}, {256, 16}, {512, 16}, {512, 32}, {128, 8}};
constexpr int kNumTube = sizeof(kTube) / sizeof(kTube[0]);

template <typename T, bool EXT>
const void* tube_func(int v) {
  switch (v) {
    case 0: return (const void*)&k_step_tubes<T, 256, EXT>;
    case 1: return (const void*)&k_step_tubes<T, 256, EXT>;
    case 2: return (const void*)&k_step_tubes<T, 512, EXT>;
    case 3: return (const void*)&k_step_tubes<T, 512, EXT>;
    case 4: return (const void*)&k_step_tubes<T, 128, EXT>;
  }
  return nullptr;
}

int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T, int BX, int BY, int CZ, bool EXT, bool NTS>
void lat_launch_stores(bool diag, dim3 grid, dim3 block, unsigned lds, const void* src, void* dst,
                       const LatticeGeom& g, double* partials, unsigned long long* bad,
                       hipStream_t s) {
  if (diag)
    hipLaunchKernelGGL((k_step_lattice<T, BX, BY, CZ, true, EXT, NTS>), grid, block, lds, s,
                       (const T*)src, (T*)dst, g, partials, bad);
  else
    hipLaunchKernelGGL((k_step_lattice<T, BX, BY, CZ, false, EXT, NTS>), grid, block, lds, s,
                       (const T*)src, (T*)dst, g, partials, bad);
}

template <typename T, int BX, int BY, int CZ, bool EXT>
hipError_t lat_launch(bool diag, const void* src, void* dst, const LatticeGeom& g,
                      double* partials, unsigned long long* bad, hipStream_t s,
                      unsigned lds = 0) {
  dim3 block(BX, BY, 1);
  dim3 grid((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY, (g.nz + CZ - 1) / CZ);
  if (g.cached_store)
    lat_launch_stores<T, BX, BY, CZ, EXT, false>(diag, grid, block, lds, src, dst, g, partials,
                                                 bad, s);
  else
    lat_launch_stores<T, BX, BY, CZ, EXT, true>(diag, grid, block, lds, src, dst, g, partials,
                                                bad, s);
  return hipGetLastError();
}

template <typename T, bool EXT>
hipError_t lat_dispatch(int v, bool diag, const void* src, void* dst, const LatticeGeom& g,
                        double* partials, unsigned long long* bad, hipStream_t s) {
  switch (v) {
    case 0: return lat_launch<T, 64, 1, 1, EXT>(diag, src, dst, g, partials, bad, s);
    case 1: return lat_launch<T, 64, 4, 1, EXT>(diag, src, dst, g, partials, bad, s);
    case 2: return lat_launch<T, 128, 2, 1, EXT>(diag, src, dst, g, partials, bad, s);
    case 3: return lat_launch<T, 256, 1, 1, EXT>(diag, src, dst, g, partials, bad, s);
    case 4: return lat_launch<T, 64, 4, 2, EXT>(diag, src, dst, g, partials, bad, s);
    case 5: return lat_launch<T, 256, 1, 2, EXT>(diag, src, dst, g, partials, bad, s);
    case 6: return lat_launch<T, 128, 2, 4, EXT>(diag, src, dst, g, partials, bad, s);
    case 7: return lat_launch<T, 256, 1, 4, EXT>(diag, src, dst, g, partials, bad, s);
    case 8: return lat_launch<T, 128, 2, 1, EXT>(diag, src, dst, g, partials, bad, s, kOcc3Lds);
    case 9: return lat_launch<T, 256, 1, 1, EXT>(diag, src, dst, g, partials, bad, s, kOcc3Lds);
  }
  return hipErrorInvalidValue;
}

template <typename T, bool EXT>
const void* mem_func(int v) {
  switch (v) {
    case 0: return (const void*)&k_step_members<T, 256, 1, EXT>;
    case 1: return (const void*)&k_step_members<T, 512, 1, EXT>;
    case 2: return (const void*)&k_step_members<T, 256, 2, EXT>;
    case 3: return (const void*)&k_step_members<T, 512, 2, EXT>;
  }
  return nullptr;
}

// Total of the inadmissible-cell slots (count_bad) into *out: one block of
// kBadSlots threads.
__global__ __launch_bounds__(kBadSlots) void k_sum_bad(const unsigned long long* __restrict__ slots,
                                                        unsigned long long* __restrict__ out) {
  __shared__ unsigned long long sh[kBadSlots];
  sh[threadIdx.x] = slots[(size_t)threadIdx.x * kBadStride];
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int k = 0; k < kBadSlots; ++k) t += sh[k];
    *out = t;
  }
}

}  // namespace

int num_lattice_variants() { return kNumLat; }
int num_segment_variants() { return kNumSeg; }
int num_tube_variants() { return kNumTube; }
TubeVariant tube_variant(int i) { return kTube[i]; }

hipError_t tube_kernel(int precision, int v, bool ext, const void** func, dim3* block) {
  if (v < 0 || v >= kNumTube) return hipErrorInvalidValue;
  if (ext)
    *func = precision ? tube_func<float, true>(v) : tube_func<double, true>(v);
  else
    *func = precision ? tube_func<float, false>(v) : tube_func<double, false>(v);
  *block = dim3(kTube[v].nt, 1, 1);
  return hipSuccess;
}

const char* tube_kernel_name(int precision, int v) {
  static const char* n32[] = {"k_step_tubes<float,256>/h8", "k_step_tubes<float,256>/h16",
                              "k_step_tubes<float,512>/h16", "k_step_tubes<float,512>/h32",
                              "k_step_tubes<float,128>/h8"};
  static const char* n64[] = {"k_step_tubes<double,256>/h8", "k_step_tubes<double,256>/h16",
                              "k_step_tubes<double,512>/h16", "k_step_tubes<double,512>/h32",
                              "k_step_tubes<double,128>/h8"};
  if (v < 0 || v >= kNumTube) return "?";
  return precision ? n32[v] : n64[v];
}
MemberVariant segment_variant(int i) { return kSeg[i]; }

hipError_t segment_kernel(int precision, int v, const void** func, dim3* block) {
  if (v < 0 || v >= kNumSeg) return hipErrorInvalidValue;
  *func = precision ? seg_func<float>(v) : seg_func<double>(v);
  *block = dim3(kSeg[v].nt, 1, 1);
  return hipSuccess;
}

const char* segment_kernel_name(int precision, int v) {
  static const char* n32[] = {"k_step_segments<float,256,1>", "k_step_segments<float,256,2>",
                              "k_step_segments<float,512,1>", "k_step_segments<float,128,4>",
                              "k_step_segments<float,256,4>"};
  static const char* n64[] = {"k_step_segments<double,256,1>", "k_step_segments<double,256,2>",
                              "k_step_segments<double,512,1>", "k_step_segments<double,128,4>",
                              "k_step_segments<double,256,4>"};
  if (v < 0 || v >= kNumSeg) return "?";
  return precision ? n32[v] : n64[v];
}
LatticeVariant lattice_variant(int i) { return kLat[i]; }
int num_member_variants() { return kNumMem; }
MemberVariant member_variant(int i) { return kMem[i]; }

int lattice_partials(int v, const LatticeGeom& g) {
  const LatticeVariant lv = kLat[v];
  return ((g.nx + lv.bx - 1) / lv.bx) * ((g.ny + lv.by - 1) / lv.by) *
         ((g.nz + lv.cz - 1) / lv.cz);
}

const char* lattice_kernel_name(int precision, int v) {
  static const char* n32[] = {"k_step_lattice<float,64,1,1>",  "k_step_lattice<float,64,4,1>",
                              "k_step_lattice<float,128,2,1>", "k_step_lattice<float,256,1,1>",
                              "k_step_lattice<float,64,4,2>",  "k_step_lattice<float,256,1,2>",
                              "k_step_lattice<float,128,2,4>", "k_step_lattice<float,256,1,4>",
                              "k_step_lattice<float,128,2,1>/w3",
                              "k_step_lattice<float,256,1,1>/w3"};
  static const char* n64[] = {
      "k_step_lattice<double,64,1,1>",     "k_step_lattice<double,64,4,1>",
      "k_step_lattice<double,128,2,1>",    "k_step_lattice<double,256,1,1>",
      "k_step_lattice<double,64,4,2>",     "k_step_lattice<double,256,1,2>",
      "k_step_lattice<double,128,2,4>",    "k_step_lattice<double,256,1,4>",
      "k_step_lattice<double,128,2,1>/w3", "k_step_lattice<double,256,1,1>/w3"};
  if (v < 0 || v >= kNumLat) return "?";
  return precision ? n32[v] : n64[v];
}

const char* member_kernel_name(int precision, int v) {
  static const char* n32[] = {"k_step_members<float,256,1>", "k_step_members<float,512,1>",
                              "k_step_members<float,256,2>", "k_step_members<float,512,2>"};
  static const char* n64[] = {"k_step_members<double,256,1>", "k_step_members<double,512,1>",
                              "k_step_members<double,256,2>", "k_step_members<double,512,2>"};
  if (v < 0 || v >= kNumMem) return "?";
  return precision ? n32[v] : n64[v];
}

hipError_t launch_member_refs(const MemberDesc* descs, int n_members, const double* n0,
                              const double* eps0, const double* u0, int64_t ncells,
                              double* parts, hipStream_t s) {
  hipLaunchKernelGGL(k_member_ref_parts, dim3(kRefBlocks, n_members), dim3(256), 0, s, descs, n0,
                     eps0, u0, ncells, parts);
  hipLaunchKernelGGL(k_member_ref_final, dim3(n_members), dim3(64), 0, s,
                     const_cast<MemberDesc*>(descs), (const double*)parts);
  return hipGetLastError();
}

hipError_t launch_validate(const double* n0, const double* eps0, const double* u0,
                           int64_t ncells, int planar, const MemberDesc* descs, int n_members,
                           unsigned long long* count, hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3(grid_for(ncells)), dim3(256), 0, s, n0, eps0, u0, ncells,
                     planar, descs, n_members, count);
  return hipGetLastError();
}

hipError_t launch_init(int precision, void* state, int64_t cs, const MemberDesc* descs,
                       int n_members, const double* n0, const double* eps0, const double* u0,
                       int64_t ncells, hipStream_t s) {
  dim3 grid(grid_for(ncells));
  if (precision)
    hipLaunchKernelGGL(k_init<float>, grid, dim3(256), 0, s, (float*)state, cs, descs,
                       n_members, n0, eps0, u0, ncells);
  else
    hipLaunchKernelGGL(k_init<double>, grid, dim3(256), 0, s, (double*)state, cs, descs,
                       n_members, n0, eps0, u0, ncells);
  return hipGetLastError();
}

hipError_t launch_step_lattice(int precision, int v, bool diag, bool ext, const void* src,
                               void* dst, const LatticeGeom& g, double* partials,
                               unsigned long long* bad, hipStream_t s) {
  if (precision)
    return ext ? lat_dispatch<float, true>(v, diag, src, dst, g, partials, bad, s)
              : lat_dispatch<float, false>(v, diag, src, dst, g, partials, bad, s);
  return ext ? lat_dispatch<double, true>(v, diag, src, dst, g, partials, bad, s)
            : lat_dispatch<double, false>(v, diag, src, dst, g, partials, bad, s);
}

hipError_t member_kernel(int precision, int v, bool ext, const void** func, dim3* block) {
  if (v < 0 || v >= kNumMem) return hipErrorInvalidValue;
  if (ext)
    *func = precision ? mem_func<float, true>(v) : mem_func<double, true>(v);
  else
    *func = precision ? mem_func<float, false>(v) : mem_func<double, false>(v);
  *block = dim3(kMem[v].nt, 1, 1);
  return hipSuccess;
}

hipError_t launch_step_members(int precision, int v, int n_members, const MemberLaunch& a,
                               hipStream_t s) {
  const void* f;
  dim3 block;
  hipError_t e = member_kernel(precision, v, false, &f, &block);
  if (e != hipSuccess) return e;
  void* args[] = {const_cast<MemberLaunch*>(&a)};
  return hipLaunchKernel(f, dim3(n_members), block, args, 0, s);
}

hipError_t launch_export(int precision, const void* state, int64_t cs, const MemberDesc* descs,
                         int n_members, int64_t ncells, double* n, double* eps, double* P,
                         double* gamma, double* u, double* partials, int nparts,
                         hipStream_t s) {
  if (precision)
    hipLaunchKernelGGL(k_export<float>, dim3(nparts), dim3(256), 0, s, (const float*)state, cs,
                       descs, n_members, ncells, n, eps, P, gamma, u, partials);
  else
    hipLaunchKernelGGL(k_export<double>, dim3(nparts), dim3(256), 0, s, (const double*)state,
                       cs, descs, n_members, ncells, n, eps, P, gamma, u, partials);
  return hipGetLastError();
}

hipError_t launch_population_planes(int precision, const void* state, int64_t cs,
                                    const MemberDesc* descs, int n_members, int64_t ncells,
                                    int p0, int np, double* out, hipStream_t s) {
  dim3 grid(grid_for(ncells));
  if (precision)
    hipLaunchKernelGGL(k_population_planes<float>, grid, dim3(256), 0, s, (const float*)state,
                       cs, descs, n_members, ncells, p0, np, out);
  else
    hipLaunchKernelGGL(k_population_planes<double>, grid, dim3(256), 0, s,
                       (const double*)state, cs, descs, n_members, ncells, p0, np, out);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nparts, double* out5, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, nparts, out5);
  return hipGetLastError();
}

hipError_t launch_sum_bad(const unsigned long long* slots, unsigned long long* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_sum_bad, dim3(1), dim3(kBadSlots), 0, s, slots, out);
  return hipGetLastError();
}

}  // namespace rlb
