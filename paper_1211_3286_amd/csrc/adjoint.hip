// Tape and adjoint of the g update (rlb_grad).
//
// Forward: rlb_step keeps g every K steps (checkpoints). Reverse: for each
// segment [kK, kK + K), last first, the g states are recomputed from the
// checkpoint with a g-only step that is bit-identical to the forward (g never
// reads f), then one adjoint kernel per step runs backwards. Each adjoint
// kernel reads, per cell, the 19 forward populations it pulled at that step
// (from the recomputed state), gathers the 19 adjoint populations of the cells
// that pulled from it (the transpose of streaming: one source per population
// in the interior, up to four at clamped corners, never an atomic), applies
// the transposed collision Jacobian (adjoint_cell.hpp) and writes 19 values:
// 3 x 19 populations of traffic per cell-step. dL/dtau is accumulated in FP64
// per block across all steps and reduced once at the end. The whole reverse
// sweep is one HIP graph in which the recomputation of the next segment runs
// beside the reverse steps of the current one (two segment buffers).

#include <hip/hip_runtime.h>

#include <algorithm>

#include "adjoint.hpp"
#include "adjoint_cell.hpp"
#include "device_util.hpp"

namespace rlb {

namespace {

size_t al(size_t v) { return (v + 255) / 256 * 256; }

int grid_of(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

// What the reverse-sweep kernels read of the lattice (a small argument, held
// in scalar registers): shape, boundaries, relaxation rates and reference.
struct AdjGeom {
  int32_t nx, ny, nz, bcx, bcy, bcz;
  Rates rt;
  Ref ref;
};

AdjGeom adj_geom(const MemberDesc& d) {
  AdjGeom g;
  g.nx = d.nx;
  g.ny = d.ny;
  g.nz = d.nz;
  g.bcx = d.bcx;
  g.bcy = d.bcy;
  g.bcz = d.bcz;
  g.rt = d.rt;
  g.ref = d.ref;
  return g;
}

template <typename G>
__device__ __forceinline__ void decompose(int c, const G& d, int& x, int& y, int& z) {
  x = c % d.nx;
  const int yz = c / d.nx;
  y = yz % d.ny;
  z = yz / d.ny;
}

// The step kernels' geometry: each wave takes 64 consecutive x-cells of one
// row (y, z), a block kRows rows, one cell per thread. The row index is
// uniform in a wave, so (y, z) come from a scalar division and no cell index
// is divided; with no loop over cells the reverse step fits 101 VGPRs (4
// waves per SIMD: a 512 x 512 step in one round of waves).
constexpr int kRows = 4;
constexpr int64_t kMaxGridY = 65535;

// The 8 XCDs of the chip take the blocks of a launch in turn (block b on XCD
// b mod 8), each XCD behind its own L2. Taken as launched, the 8 blocks of a
// 512-cell row went to 8 XCDs: each XCD kept a 64-cell column strip, and the
// line at each edge of a strip, which the x-shifted pulls of the waves on
// both sides share, was fetched by two XCDs. The kernels renumber their
// blocks so that each XCD takes one contiguous run of row blocks, a band of
// whole rows: no row is split over XCDs.
constexpr unsigned kXcds = 8;

dim3 row_grid(const AdjGeom& g) {
  const int64_t rows = (int64_t)g.ny * g.nz;
  const int64_t nrb = (rows + kRows - 1) / kRows;
  const int64_t gy = std::min(nrb, kMaxGridY);
  return dim3((unsigned)((g.nx + 63) / 64), (unsigned)gy, (unsigned)((nrb + gy - 1) / gy));
}

int64_t row_blocks(const AdjGeom& g) {
  const dim3 r = row_grid(g);
  return (int64_t)r.x * r.y * r.z;
}

// This thread's cell: x, and its row r = y + ny z (uniform in its wave).
// Launched block b, on XCD j = b mod 8, is the (b / 8)-th of that XCD's run
// of logical blocks: XCD j takes q + (j < rem) of the nb = 8q + rem blocks,
// starting at jq + min(j, rem). The renumbering is one to one for any nb.
__device__ __forceinline__ void row_cell(int& x, int& r) {
  const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
  const unsigned b = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const unsigned j = b % kXcds, q = nb / kXcds, rem = nb % kXcds;
  const unsigned lb = j * q + (j < rem ? j : rem) + b / kXcds;
  x = (int)((lb % gridDim.x) * 64 + threadIdx.x);
  r = __builtin_amdgcn_readfirstlane((int)((lb / gridDim.x) * kRows + threadIdx.y));
}

// Cells y with src(y, e) = c along one axis (the pull source is y - e,
// wrapped or clamped): one in the interior, up to two at a clamped end.
__device__ __forceinline__ int preimages(int c, int e, int N, int bc, int (&out)[2]) {
  if (e == 0) {
    out[0] = c;
    return 1;
  }
  int s = c + e;
  if (bc == 0) {
    if (s < 0) s += N;
    if (s >= N) s -= N;
    out[0] = s;
    return 1;
  }
  int n = 0;
  if (s >= 0 && s <= N - 1) out[n++] = s;
  if (e > 0 && c == 0) out[n++] = 0;
  if (e < 0 && c == N - 1) out[n++] = N - 1;
  return n;
}

// Transposed streaming: adjoint of the pre-collision populations of the cells
// that pulled population a from cell (x, y, z), summed. Away from clamped
// faces that cell is x + e_a, the pull source of the opposite population
// (e_opp = -e_a), so the gather is 19 plain loads; cells on a clamped face
// walk the preimage sets per axis.
__device__ __forceinline__ int opposite(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }

template <typename T, typename G>
__device__ __forceinline__ void gather_adjoint(const T* __restrict__ adj, int64_t cs, int x, int y,
                                               int z, const G& d, T (&gb)[19]) {
  const bool face = (d.bcx && (x == 0 || x == d.nx - 1)) ||
                    (d.bcy && (y == 0 || y == d.ny - 1)) ||
                    (d.bcz && (z == 0 || z == d.nz - 1));
  if (!face) {
    uint32_t off[19], self;
    pull_offsets(x, y, z, d.nx, d.ny, d.nz, d.bcx, d.bcy, d.bcz, 0u, (uint32_t)sizeof(T), off,
                 self);
#pragma unroll
    for (int a = 0; a < 19; ++a) gb[a] = ld(adj + (int64_t)a * cs, off[opposite(a)]);
    return;
  }
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    int px[2], py[2], pz[2];
    const int nxp = preimages(x, ex(a), d.nx, d.bcx, px);
    const int nyp = preimages(y, ey(a), d.ny, d.bcy, py);
    const int nzp = preimages(z, ez(a), d.nz, d.bcz, pz);
    T s = T(0.0);
    for (int k = 0; k < nzp; ++k)
      for (int j = 0; j < nyp; ++j)
        for (int i = 0; i < nxp; ++i)
          s += adj[(int64_t)a * cs + ((int64_t)pz[k] * d.ny + py[j]) * d.nx + px[i]];
    gb[a] = s;
  }
}

// One DPP exchange of a double between the lanes of a row of 16 (CTRL a
// permutation within the row, so every lane receives a value).
template <int CTRL>
__device__ __forceinline__ double dpp_row(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum of a double over the 64 lanes of a wave (all lanes active), uniform in
// the wave: four DPP exchanges make every lane of a row of 16 hold the row's
// sum (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror,
// row_mirror), then the four row sums are read out. VALU work only: no LDS
// round trips, which matter when every wave of a single-round launch reduces
// at the same time.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_row<0xB1>(v);
  v += dpp_row<0x4E>(v);
  v += dpp_row<0x141>(v);
  v += dpp_row<0x140>(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// g-only forward step between g-plane buffers (recomputation of a segment).
template <typename T>
__global__ __launch_bounds__(256) void k_gstep(const T* __restrict__ src, T* __restrict__ dst,
                                               int64_t cs, AdjGeom d) {
  const uint32_t esz = sizeof(T);
  int x, r;
  row_cell(x, r);
  if (x < d.nx && r < d.ny * d.nz) {
    const int y = r % d.ny, z = r / d.ny;
    uint32_t off[19], self;
    pull_offsets(x, y, z, d.nx, d.ny, d.nz, d.bcx, d.bcy, d.bcz, 0u, esz, off, self);
    T g[19];
#pragma unroll
    for (int a = 0; a < 19; ++a) g[a] = ld(src + (int64_t)a * cs, off[a]);
    collide_g_only(g, d.rt, d.ref);
#pragma unroll
    for (int a = 0; a < 19; ++a) st(dst + (int64_t)a * cs, self, g[a]);
  }
}

// dL/dg* of the final state from dL/du, dL/deps.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_loss(const T* __restrict__ state, int64_t cs,
                                                  MemberDesc d, const double* __restrict__ dLdu,
                                                  const double* __restrict__ dLdeps,
                                                  T* __restrict__ out) {
  const int64_t nc = d.ncells;
  for (int c = blockIdx.x * 256 + threadIdx.x; c < d.ncells; c += gridDim.x * 256) {
    T g[19], gb[19];
#pragma unroll
    for (int a = 0; a < 19; ++a) g[a] = state[(int64_t)a * cs + c];
    loss_adjoint(g, d.ref, dLdu[c], dLdu[nc + c], dLdu[2 * nc + c], dLdeps[c], gb);
#pragma unroll
    for (int a = 0; a < 19; ++a) out[(int64_t)a * cs + c] = gb[a];
  }
}

// One reverse step. state: g*(t) (the step's input); adj_in: either the
// adjoint of g*(t+1) (GATHER = false, straight from the loss) or the
// pre-collision adjoint of step t+1 (GATHER = true, transposed streaming
// applied here). adj_out: pre-collision adjoint of step t. Row geometry of
// k_gstep; dL/dtau partials per block.
template <typename T, bool GATHER>
__global__ __launch_bounds__(256) void k_adj_step(const T* __restrict__ state,
                                                  const T* __restrict__ adj_in,
                                                  T* __restrict__ adj_out, int64_t cs, AdjGeom d,
                                                  double* __restrict__ partials) {
  const uint32_t esz = sizeof(T);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int x, r;
  row_cell(x, r);
  if (x < d.nx && r < d.ny * d.nz) {
    const int y = r % d.ny, z = r / d.ny;
    uint32_t off[19], self;
    pull_offsets(x, y, z, d.nx, d.ny, d.nz, d.bcx, d.bcy, d.bcz, 0u, esz, off, self);
    AdjPrep<T> pr;
    {
      T g[19];
#pragma unroll
      for (int a = 0; a < 19; ++a) g[a] = ld(state + (int64_t)a * cs, off[a]);
      adjoint_prepare(g, d.ref, pr);
    }
    T gb[19];
    if (GATHER) {
      gather_adjoint(adj_in, cs, x, y, z, d, gb);
    } else {
      const int64_t c = (int64_t)r * d.nx + x;
#pragma unroll
      for (int a = 0; a < 19; ++a) gb[a] = adj_in[(int64_t)a * cs + c];
    }
    adjoint_apply(pr, gb, d.rt, acc);
#pragma unroll
    for (int a = 0; a < 19; ++a) st(adj_out + (int64_t)a * cs, self, gb[a]);
  }
  // The block's four dL/dtau sums: one per wave by DPP, then thread 0 adds
  // the kRows waves' sums into the block's own partials slot.
  __shared__ double sh[kRows][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = wave_sum(acc[q]);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 4; ++q) sh[threadIdx.y][q] = acc[q];
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    double* p =
        partials + (((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * 5;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kRows; ++w) s += sh[w][q];
      p[q] += s;
    }
  }
}

// dL/deps0, dL/du0 from the adjoint of the initial state.
template <typename T, bool GATHER>
__global__ __launch_bounds__(256) void k_adj_init(const T* __restrict__ adj_in, int64_t cs,
                                                  MemberDesc d, const double* __restrict__ f0,
                                                  double* __restrict__ deps0,
                                                  double* __restrict__ du0) {
  const int64_t nc = d.ncells;
  for (int c = blockIdx.x * 256 + threadIdx.x; c < d.ncells; c += gridDim.x * 256) {
    T gb[19];
    if (GATHER) {
      int x, y, z;
      decompose(c, d, x, y, z);
      gather_adjoint(adj_in, cs, x, y, z, d, gb);
    } else {
#pragma unroll
      for (int a = 0; a < 19; ++a) gb[a] = adj_in[(int64_t)a * cs + c];
    }
    double de, dx, dy, dz;
    init_adjoint(gb, f0[c], f0[nc + c], f0[2 * nc + c], f0[3 * nc + c], de, dx, dy, dz);
    deps0[c] = de;
    du0[c] = dx;
    du0[nc + c] = dy;
    du0[2 * nc + c] = dz;
  }
}

__global__ __launch_bounds__(256) void k_sum_parts(const double* parts, int n, double* out) {
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < n; j += 256)
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] += parts[(int64_t)j * 5 + k];
  block_sum5<256>(v, threadIdx.x);
  if (threadIdx.x == 0)
    for (int k = 0; k < 5; ++k) out[k] = v[k];
}

void release_graph(Tape& t) {
  if (t.graph_exec) (void)hipGraphExecDestroy(t.graph_exec);
  if (t.graph) (void)hipGraphDestroy(t.graph);
  t.graph_exec = nullptr;
  t.graph = nullptr;
  t.graph_steps = -1;
}

// Adds one kernel node after the given dependencies.
template <typename... A>
hipError_t add_node(hipGraph_t g, hipGraphNode_t* out, const hipGraphNode_t* deps, int ndeps,
                    const void* func, dim3 grid, dim3 block, A... args) {
  void* params[] = {(void*)&args...};
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(func);
  kp.gridDim = grid;
  kp.blockDim = block;
  kp.sharedMemBytes = 0;
  kp.kernelParams = params;
  kp.extra = nullptr;
  return hipGraphAddKernelNode(out, g, ndeps ? deps : nullptr, ndeps, &kp);
}

// The reverse sweep over every checkpointed segment, last first, as one HIP
// graph of kernel nodes: per segment k, the g-only recomputation of its
// states from checkpoint k (chain G(k)), then one reverse step per step of
// the segment (chain R(k)). Segments alternate between two state buffers, so
// that G(k-1) runs beside R(k), as a parallel branch of the graph: G(k-1)
// waits only for R(k+1), the last reader of its buffer, and R(k) for G(k)
// and R(k+1). The graph depends only on the step count and the tape's
// buffers: it is built once per step count and kept with the tape.
template <typename T>
rlb_status chain_graph(Tape& t, const GradContext& c) {
  const TapeLayout& L = t.L;
  const AdjGeom d = adj_geom(c.desc);
  const int64_t cs = c.cs;
  const int64_t T_steps = c.steps;
  const int K = L.K;
  const dim3 grid(row_grid(d)), block(64, kRows);
  auto ckpt = [&](int64_t k) { return (const T*)(t.base + L.off_ckpt + (size_t)k * L.gbytes); };
  auto seg = [&](int64_t k, int64_t j) {
    return (T*)(t.base + L.off_seg + (size_t)((k & 1) * K + j) * L.gbytes);
  };
  T* adj[2] = {(T*)(t.base + L.off_adj), (T*)(t.base + L.off_adj + L.gbytes)};
  double* parts = (double*)(t.base + L.off_tparts);
  hipGraph_t g = nullptr;
  if (hipGraphCreate(&g, 0) != hipSuccess) return RLB_E_DEVICE;
  hipError_t e = hipSuccess;
  // G(k) after dep (null: no dependency); *last = its last node (null when
  // the segment has a single step and nothing to recompute)
  auto add_G = [&](int64_t k, hipGraphNode_t dep, hipGraphNode_t* last) {
    const int64_t t0 = k * K;
    const int64_t t1 = std::min<int64_t>(t0 + K, T_steps);
    const T* src = ckpt(k);
    hipGraphNode_t prev = dep;
    *last = nullptr;
    for (int64_t tt = t0 + 1; tt < t1 && e == hipSuccess; ++tt) {
      T* dst = seg(k, tt - t0);
      hipGraphNode_t n;
      e = add_node(g, &n, &prev, prev ? 1 : 0, (const void*)&k_gstep<T>, grid, block, src, dst,
                   cs, d);
      prev = *last = n;
      src = dst;
    }
  };
  int cur = 0;
  bool gathered = false;
  const int64_t kmax = (T_steps - 1) / K;
  hipGraphNode_t lastG = nullptr, lastR = nullptr;
  add_G(kmax, nullptr, &lastG);
  for (int64_t k = kmax; k >= 0 && e == hipSuccess; --k) {
    const int64_t t0 = k * K;
    const int64_t t1 = std::min<int64_t>(t0 + K, T_steps);
    hipGraphNode_t nextG = nullptr;
    if (k > 0) add_G(k - 1, lastR, &nextG);  // beside R(k): after R(k+1) only
    hipGraphNode_t deps[2];
    int nd = 0;
    if (lastG) deps[nd++] = lastG;
    if (lastR) deps[nd++] = lastR;
    hipGraphNode_t prev = nullptr;
    for (int64_t tt = t1 - 1; tt >= t0 && e == hipSuccess; --tt) {
      const T* st = (tt == t0) ? ckpt(k) : (const T*)seg(k, tt - t0);
      const T* in = adj[cur];
      T* out = adj[1 - cur];
      const void* f = gathered ? (const void*)&k_adj_step<T, true>
                               : (const void*)&k_adj_step<T, false>;
      hipGraphNode_t n;
      e = prev ? add_node(g, &n, &prev, 1, f, grid, block, st, in, out, cs, d, parts)
               : add_node(g, &n, deps, nd, f, grid, block, st, in, out, cs, d, parts);
      prev = n;
      cur = 1 - cur;
      gathered = true;
    }
    lastR = prev;
    lastG = nextG;
  }
  hipGraphExec_t x = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return RLB_E_DEVICE;
  }
  release_graph(t);
  t.graph = g;
  t.graph_exec = x;
  t.graph_steps = T_steps;
  return RLB_OK;
}

template <typename T>
rlb_status run_grad(Tape& t, const GradContext& c, const double* dLdu, const double* dLdeps,
                    double dL_dtau[3], double* deps0, double* du0) {
  const TapeLayout& L = t.L;
  const MemberDesc d = c.desc;
  const int64_t cs = c.cs;
  const int64_t T_steps = c.steps;
  hipStream_t s = c.stream;
  const dim3 grid(grid_of(c.ncells)), block(256);
  const int nparts = (int)row_blocks(adj_geom(d));
  T* adj[2] = {(T*)(t.base + L.off_adj), (T*)(t.base + L.off_adj + L.gbytes)};
  const double* f0 = (const double*)(t.base + L.off_fields);
  double* parts = (double*)(t.base + L.off_tparts);
  if (T_steps > 0 && (!t.graph_exec || t.graph_steps != T_steps)) {
    const rlb_status st = chain_graph<T>(t, c);
    if (st != RLB_OK) return st;
  }
  if (hipMemsetAsync(parts, 0, sizeof(double) * 5 * (size_t)nparts, s) != hipSuccess)
    return RLB_E_DEVICE;
  const T* final_g = (const T*)((const char*)c.state + 19 * (size_t)cs * sizeof(T));
  hipLaunchKernelGGL(k_adj_loss<T>, grid, block, 0, s, final_g, cs, d, dLdu, dLdeps, adj[0]);
  if (T_steps > 0 && hipGraphLaunch(t.graph_exec, s) != hipSuccess) return RLB_E_DEVICE;
  // the chain's last reverse step wrote adj[T_steps & 1]
  const int cur = (int)(T_steps & 1);
  if (T_steps > 0)
    hipLaunchKernelGGL((k_adj_init<T, true>), grid, block, 0, s, adj[cur], cs, d, f0, deps0, du0);
  else
    hipLaunchKernelGGL((k_adj_init<T, false>), grid, block, 0, s, adj[cur], cs, d, f0, deps0,
                       du0);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, parts, nparts, c.sums_out);
  if (hipGetLastError() != hipSuccess) return RLB_E_DEVICE;
  double h[5];
  if (hipMemcpyAsync(h, c.sums_out, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return RLB_E_DEVICE;
  // groups: v, e, eps, q (q folds into v when the ghost rows follow tau_v)
  dL_dtau[0] = h[0] + (c.tau_q_tied ? h[3] : 0.0);
  dL_dtau[1] = h[1];
  dL_dtau[2] = h[2];
  return RLB_OK;
}

}  // namespace

TapeLayout tape_layout(int nx, int ny, int nz, int64_t cs, size_t esz, int K, int tape_steps,
                       int max_parts) {
  TapeLayout L;
  const int64_t ncells = (int64_t)nx * ny * nz;
  AdjGeom g{};
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  L.K = K;
  L.gbytes = 19 * (size_t)cs * esz;
  L.n_ckpt = tape_steps / K + 1;
  L.max_parts = (int)std::max<int64_t>(max_parts, row_blocks(g));  // reverse-step partials
  size_t o = 0;
  L.off_ckpt = o;
  o = al(o + L.gbytes * L.n_ckpt);
  L.off_seg = o;  // two segments' states: the one reversed, the next recomputed
  o = al(o + L.gbytes * 2 * (size_t)K);
  L.off_adj = o;
  o = al(o + 2 * L.gbytes);
  L.off_fields = o;
  o = al(o + sizeof(double) * 4 * (size_t)ncells);
  L.off_tparts = o;
  o = al(o + sizeof(double) * 5 * (size_t)L.max_parts);
  L.total = o;
  return L;
}

rlb_status tape_init(Tape& t, const TapeLayout& L, char* base, int precision, int64_t ncells,
                     int64_t cs, int K, int tape_steps, const double* n0, const double* eps0,
                     const double* u0, const void* state, hipStream_t s) {
  (void)n0;
  (void)K;
  (void)tape_steps;
  t.base = base;
  t.L = L;
  t.precision = precision;
  t.ncells = ncells;
  t.cs = cs;
  double* f = (double*)(base + L.off_fields);
  if (hipMemcpyAsync(f, eps0, sizeof(double) * ncells, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return RLB_E_DEVICE;
  if (hipMemcpyAsync(f + ncells, u0, sizeof(double) * 3 * ncells, hipMemcpyDeviceToDevice, s) !=
      hipSuccess)
    return RLB_E_DEVICE;
  return tape_checkpoint(t, 0, state, s);
}

rlb_status tape_checkpoint(Tape& t, int64_t idx, const void* state, hipStream_t s) {
  if (idx < 0 || idx >= t.L.n_ckpt) return RLB_E_STATE;
  const char* g = (const char*)state + t.L.gbytes;  // 19 f planes precede the g planes
  char* dst = t.base + t.L.off_ckpt + (size_t)idx * t.L.gbytes;
  return hipMemcpyAsync(dst, g, t.L.gbytes, hipMemcpyDeviceToDevice, s) == hipSuccess
             ? RLB_OK
             : RLB_E_DEVICE;
}

rlb_status tape_grad(Tape& t, const GradContext& c, const double* dL_du, const double* dL_deps,
                     double dL_dtau[3], double* dL_deps0, double* dL_du0, int io_on_device) {
  if (!t.base) return RLB_E_STATE;
  const int64_t nc = c.ncells;
  const double *du = dL_du, *de = dL_deps;
  double *oe = dL_deps0, *ou = dL_du0;
  if (!io_on_device) {
    double* st = c.stage;
    if (hipMemcpyAsync(st, dL_du, sizeof(double) * 3 * nc, hipMemcpyHostToDevice, c.stream) !=
            hipSuccess ||
        hipMemcpyAsync(st + 3 * nc, dL_deps, sizeof(double) * nc, hipMemcpyHostToDevice,
                       c.stream) != hipSuccess)
      return RLB_E_DEVICE;
    du = st;
    de = st + 3 * nc;
    oe = st + 4 * nc;
    ou = st + 5 * nc;
  }
  rlb_status r = c.precision ? run_grad<float>(t, c, du, de, dL_dtau, oe, ou)
                             : run_grad<double>(t, c, du, de, dL_dtau, oe, ou);
  if (r != RLB_OK) return r;
  if (!io_on_device) {
    if (hipMemcpyAsync(dL_deps0, oe, sizeof(double) * nc, hipMemcpyDeviceToHost, c.stream) !=
            hipSuccess ||
        hipMemcpyAsync(dL_du0, ou, sizeof(double) * 3 * nc, hipMemcpyDeviceToHost, c.stream) !=
            hipSuccess ||
        hipStreamSynchronize(c.stream) != hipSuccess)
      return RLB_E_DEVICE;
  }
  return RLB_OK;
}

void tape_release(Tape& t) {
  release_graph(t);
  t.base = nullptr;
}

}  // namespace rlb
