// Host-side interfaces between the C ABI (api.cpp) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "cell.hpp"

namespace rlb {

// One lattice of a batch, as the kernels see it (device copy in the workspace).
struct MemberDesc {
  int64_t offset;  // first cell in the packed population planes
  int32_t nx, ny, nz;
  int32_t ncells;  // nx*ny*nz (members of the persistent path are < 2^31 cells)
  int32_t bcx, bcy, bcz;
  int32_t pad;
  Rates rt;
  Ref ref;
  Ext ext;  // eta/s relaxation times and equation of state (EXT kernels, init, export)
};

// Geometry of a single-lattice launch (the per-step fused kernel).
struct LatticeGeom {
  int32_t nx, ny, nz;
  int32_t bcx, bcy, bcz;
  int64_t cs;  // plane stride in elements
  Rates rt;
  Ref ref;
  Ext ext;  // eta/s relaxation times and equation of state (EXT kernels, init, export)
  // 1: the one-step lattice kernels store with plain (cached) stores, so that
  // a state small enough for the memory-side cache is read back from it next
  // step; 0: nontemporal stores
  int32_t cached_store;
};

struct LatticeVariant {
  int bx, by, cz;
};
struct MemberVariant {
  int nt, cpt;
};

int num_lattice_variants();
LatticeVariant lattice_variant(int i);
int num_member_variants();
MemberVariant member_variant(int i);

// Inadmissible-cell counter: kBadSlots 64-bit counters kBadStride apart (one
// 128-byte line each); a block adds its count to the slot its linear index
// picks, so that a step with many inadmissible cells does not serialise its
// atomics on one address. The host sums the slots.
constexpr int kBadSlots = 256;
constexpr int kBadStride = 16;
constexpr size_t kBadBytes = sizeof(unsigned long long) * kBadSlots * kBadStride;

__device__ __forceinline__ void count_bad(unsigned long long* bad, int n) {
  const unsigned b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  atomicAdd(bad + (size_t)kBadStride * (b & (kBadSlots - 1)), (unsigned long long)n);
}

// precision: 0 = FP64, 1 = FP32 (rlb.h).
// Partial-sum blocks per member of the reference-state pass; the partials
// buffer must hold n_members * kRefBlocks * 5 doubles.
constexpr int kRefBlocks = 64;
hipError_t launch_member_refs(const MemberDesc* descs, int n_members, const double* n0,
                              const double* eps0, const double* u0, int64_t ncells,
                              double* parts, hipStream_t s);
// planar: also count cells with u_z != 0 (D2Q9 lattices carry no z velocity);
// cells of members with a general equation of state also need eps > m n.
hipError_t launch_validate(const double* n0, const double* eps0, const double* u0,
                           int64_t ncells, int planar, const MemberDesc* descs, int n_members,
                           unsigned long long* count, hipStream_t s);
hipError_t launch_init(int precision, void* state, int64_t cs, const MemberDesc* descs,
                       int n_members, const double* n0, const double* eps0, const double* u0,
                       int64_t ncells, hipStream_t s);
// ext: the extended model (relaxation times from eta/s, general equation of state).
hipError_t launch_step_lattice(int precision, int variant, bool diag, bool ext, const void* src,
                               void* dst, const LatticeGeom& g, double* partials,
                               unsigned long long* bad, hipStream_t s);
int lattice_partials(int variant, const LatticeGeom& g);  // number of blocks
// Kernel function pointer and launch shape of the persistent member kernel
// (for graph nodes). args must outlive the launch.
struct MemberLaunch {
  const MemberDesc* descs;
  void* bufA;
  void* bufB;
  int64_t cs;
  int32_t nsteps;
  int32_t pingpong;
  int32_t diag_every;
  int32_t pad;
  int64_t step0;
  double* partials;
  unsigned long long* bad;
};
hipError_t member_kernel(int precision, int variant, bool ext, const void** func, dim3* block);

// Segmented persistent step: every member is cut into segments of whole
// z-planes, one block per segment; a segment waits (per step) for the two
// segments whose planes it pulls from. flags[s] counts the steps segment s has
// completed; all flags equal `epoch` when a launch starts.
struct Segment {
  int32_t member;
  int32_t z0, z1;       // planes [z0, z1) of the member
  int32_t left, right;  // segments owning planes z0-1 and z1 (-1: none / self)
};
struct SegLaunch {
  const MemberDesc* descs;
  const Segment* segs;
  void* bufA;
  void* bufB;
  int64_t cs;
  int32_t nsteps;
  int32_t pingpong;
  int32_t diag_every;
  int32_t spin_limit;  // polls before a wait gives up and flags an error
  int64_t step0;
  unsigned long long epoch;
  unsigned long long* flags;
  int* error;
  double* partials;
  unsigned long long* bad;
};
// Quasi-1D members (1 x 1 x L tubes) by rounds of LDS-resident steps: a block
// owns cells [own0, own1) of one tube and loads the window [win0, win0 + wlen)
// (the owned cells plus up to H halo cells per side); after h <= H steps in
// LDS the owned cells are exact and written back. Window edges are either a
// halo (validity shrinks by one cell per step), the tube's zero-gradient end,
// or a wrap when the window holds a whole periodic tube.
enum : int32_t { kEdgeHalo = 0, kEdgeClamp = 1, kEdgeWrap = 2 };
struct TubeSeg {
  int32_t member;
  int32_t own0, own1;
  int32_t win0, wlen;
  int32_t left, right;  // edge kinds
};
struct TubeRound {
  const MemberDesc* descs;
  const TubeSeg* segs;
  const void* src;
  void* dst;
  int64_t cs;
  int32_t nsteps;  // steps of this round (<= H)
  int32_t diag_every;
  int64_t step0;      // global index of the step before this round's first
  int64_t last_step;  // global index of the last step of the rlb_step call
  double* partials;
  unsigned long long* bad;
};
struct TubeVariant {
  int nt, halo;
};
int num_tube_variants();
TubeVariant tube_variant(int i);
hipError_t tube_kernel(int precision, int variant, bool ext, const void** func, dim3* block);
const char* tube_kernel_name(int precision, int variant);

int num_segment_variants();
MemberVariant segment_variant(int i);  // (threads per block, cells per thread)
hipError_t segment_kernel(int precision, int variant, const void** func, dim3* block);
const char* segment_kernel_name(int precision, int variant);
hipError_t launch_step_members(int precision, int variant, int n_members, const MemberLaunch& a,
                               hipStream_t s);
hipError_t launch_export(int precision, const void* state, int64_t cs, const MemberDesc* descs,
                         int n_members, int64_t ncells, double* n, double* eps, double* P,
                         double* gamma, double* u, double* partials, int nparts, hipStream_t s);
hipError_t launch_population_planes(int precision, const void* state, int64_t cs,
                                    const MemberDesc* descs, int n_members, int64_t ncells,
                                    int p0, int np, double* out, hipStream_t s);
hipError_t launch_reduce(const double* partials, int nparts, double* out5, hipStream_t s);
// The total of the inadmissible-cell slots into *out (device).
hipError_t launch_sum_bad(const unsigned long long* slots, unsigned long long* out,
                          hipStream_t s);
const char* lattice_kernel_name(int precision, int variant);
const char* member_kernel_name(int precision, int variant);

// D2Q9 model (kernels2d.hip): 18 planes per buffer, nz = 1. LatticeVariant
// cz is the number of cells per thread along y.
int d2q9_num_lattice_variants();
int d2q9_lattice_partials(int variant, const LatticeGeom& g);
const char* d2q9_lattice_kernel_name(int precision, int variant);
// corr: apply the correction term of Eqs. (37)-(38) (flows along y);
// ext: the extended model (relaxation times from eta/s, general equation of state).
hipError_t d2q9_launch_step_lattice(int precision, int variant, bool diag, bool corr, bool ext,
                                    const void* src, void* dst, const LatticeGeom& g,
                                    double* partials, unsigned long long* bad, hipStream_t s);
int d2q9_num_member_variants();
hipError_t d2q9_member_kernel(int precision, int variant, bool corr, bool ext, const void** func,
                              dim3* block);
const char* d2q9_member_kernel_name(int precision, int variant);
// Tile rounds of the D2Q9 lattice path (k_d2q9_tiles): one block per tile of
// ox x oy owned cells, whose window (the tile plus hx / hy halo cells a side,
// cut at zero-gradient faces; an axis no longer than the block is taken whole)
// advances nsteps <= H steps in LDS.
struct TileRound {
  const void* src;
  void* dst;
  int64_t cs;
  int32_t nx, ny, bcx, bcy;
  int32_t ox, oy;  // owned cells per tile and axis (when the axis is tiled)
  int32_t hx, hy;  // halo cells a side per axis
  int32_t nsteps, diag_every;
  int64_t step0, last_step;
  Rates rt;
  Ref ref;
  Ext ext;
  double* partials;
  unsigned long long* bad;
};
struct TileVariant {
  int tx, ty, h;  // block (= window) shape, steps per launch
};
int d2q9_num_tile_variants();
bool d2q9_tile_fits(int precision, int variant, bool corr);  // LDS of the block within 160 KB
TileVariant d2q9_tile_variant(int i);
hipError_t d2q9_launch_tiles(int precision, int variant, bool corr, bool ext, const TileRound& a,
                             dim3 grid, hipStream_t s);
const char* d2q9_tile_kernel_name(int precision, int variant);
// Strip rounds (k_d2q9_strips): TubeVariant.halo is the number of steps per
// launch; the window's halo is that many rows, twice that with the correction.
int d2q9_num_strip_variants();
TubeVariant d2q9_strip_variant(int i);
hipError_t d2q9_strip_kernel(int precision, int variant, bool corr, bool ext, const void** func,
                             dim3* block);
const char* d2q9_strip_kernel_name(int precision, int variant);
hipError_t d2q9_launch_init(int precision, void* state, int64_t cs, const MemberDesc* descs,
                            int n_members, const double* n0, const double* eps0,
                            const double* u0, int64_t ncells, hipStream_t s);
hipError_t d2q9_launch_export(int precision, const void* state, int64_t cs,
                              const MemberDesc* descs, int n_members, int64_t ncells, double* n,
                              double* eps, double* P, double* gamma, double* u,
                              double* partials, int nparts, hipStream_t s);
hipError_t d2q9_launch_population_planes(int precision, const void* state, int64_t cs,
                                         const MemberDesc* descs, int n_members, int64_t ncells,
                                         int p0, int np, double* out, hipStream_t s);

}  // namespace rlb
