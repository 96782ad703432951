// C ABI of the relativistic lattice Boltzmann library (include/rlb.h):
// argument validation, workspace carving, dispatch, graphs, autotuning.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/rlb.h"
#include "adjoint.hpp"
#include "internal.hpp"

using rlb::LatticeGeom;
using rlb::MemberDesc;

namespace {

constexpr size_t kAlign = 256;
// A single lattice at least this large takes the lattice path (one fused
// launch per step, or D2Q9 tile rounds); smaller lattices and batches take the
// persistent path (per-member kernels, segments, tube or strip rounds).
constexpr int64_t kLatticeMinCells = 16384;
// Double-buffered states up to this size are stored with plain stores.
constexpr size_t kCachedStateBytes = size_t(1) << 30;
// Pad after each population plane (see make_layout).
constexpr int64_t kPlanePadBytes = 1280;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  int64_t ncells = 0, cs = 0;
  size_t esz = 0;
  size_t off_descs = 0, off_small = 0, off_bad = 0, off_partials = 0, off_xparts = 0,
         off_buf0 = 0, off_buf1 = 0;
  size_t off_stage = 0, off_segs = 0, off_flags = 0, off_tape = 0, total = 0;
  int max_parts = 0;
  int export_parts = 0;  // blocks of the field export (its own partials region)
  int64_t max_segs = 0;  // persistent path: one segment per z-plane (D2Q9: per row) at most
  rlb::TapeLayout tape;
};

bool finite_tau(double t) { return std::isfinite(t) && t > 0.5; }

rlb_status check_members(const rlb_params* m, int32_t n, int64_t* ncells) {
  if (!m || n < 1) return RLB_E_ARG;
  int64_t tot = 0;
  for (int i = 0; i < n; ++i) {
    const rlb_params& p = m[i];
    if (p.nx < 1 || p.ny < 1 || p.nz < 1) return RLB_E_ARG;
    for (int k = 0; k < 3; ++k)
      if (p.bc[k] != RLB_PERIODIC && p.bc[k] != RLB_ZERO_GRADIENT) return RLB_E_ARG;
    const int64_t c = (int64_t)p.nx * p.ny * p.nz;
    if (c >= (int64_t(1) << 31)) return RLB_E_UNSUPPORTED;
    tot += c;
  }
  for (int i = 0; i < n; ++i) {
    const rlb_params& p = m[i];
    if (!finite_tau(p.tau_f) || !finite_tau(p.tau_v) || !finite_tau(p.tau_e) ||
        !finite_tau(p.tau_eps))
      return RLB_E_TAU;
    if (p.tau_q > 0.0 && !finite_tau(p.tau_q)) return RLB_E_TAU;
    if (std::isnan(p.tau_q)) return RLB_E_TAU;
    if (!std::isfinite(p.eta_over_s) || p.eta_over_s < 0.0) return RLB_E_ARG;
    if (!(p.eos_gamma == 0.0 || (p.eos_gamma > 1.0 && p.eos_gamma <= 2.0))) return RLB_E_ARG;
    if (!std::isfinite(p.mass) || p.mass < 0.0) return RLB_E_ARG;
    if (p.eta_over_s > 0.0) {
      if (!std::isfinite(p.kappa) || !(p.kappa > 0.0)) return RLB_E_ARG;
      if (!std::isfinite(p.dof) || !(p.dof > 0.0)) return RLB_E_ARG;
      for (double a : {p.a_f, p.a_e, p.a_eps, p.a_q})
        if (!std::isfinite(a) || a < 0.0) return RLB_E_ARG;
    }
  }
  *ncells = tot;
  return RLB_OK;
}

// The paper's equation of state P = eps/3 (Gamma 0 or 4/3, no rest mass)?
bool paper_eos(const rlb_params& p) {
  return (p.eos_gamma == 0.0 || p.eos_gamma == 4.0 / 3.0) && p.mass == 0.0;
}

bool lattice_path(int32_t n_members, int64_t ncells) {
  return n_members == 1 && ncells >= kLatticeMinCells;
}

// Velocities per distribution of a lattice kind.
int nvel(int32_t lattice) { return lattice == RLB_D2Q9 ? 9 : 19; }

// Tile geometry of a D2Q9 tile variant on an nx x ny lattice: halo cells a
// side (y doubled with the correction term), owned cells per tile and the
// grid. false when a tiled axis leaves no owned cell.
bool tile_geometry(const rlb::TileVariant& v, int nx, int ny, bool corr, rlb::TileRound& a,
                   dim3& grid) {
  a.hx = v.h;
  a.hy = corr ? 2 * v.h : v.h;
  a.ox = v.tx - 2 * a.hx;
  a.oy = v.ty - 2 * a.hy;
  if ((nx > v.tx && a.ox < 1) || (ny > v.ty && a.oy < 1)) return false;
  grid = dim3(nx <= v.tx ? 1 : (nx + a.ox - 1) / a.ox, ny <= v.ty ? 1 : (ny + a.oy - 1) / a.oy, 1);
  return true;
}

rlb_status make_layout(const rlb_params* m, int32_t n, const rlb_options* opt, Layout& L) {
  if (!opt) return RLB_E_ARG;
  if (opt->precision != RLB_FP32 && opt->precision != RLB_FP64) return RLB_E_ARG;
  if (opt->ckpt_every < 0 || opt->tape_steps < 0 || opt->diag_every < 0) return RLB_E_ARG;
  if (opt->lattice != RLB_D3Q19 && opt->lattice != RLB_D2Q9) return RLB_E_ARG;
  if (opt->correction != 0 && opt->correction != 1) return RLB_E_ARG;
  if (opt->correction && opt->lattice != RLB_D2Q9) return RLB_E_UNSUPPORTED;
  rlb_status st = check_members(m, n, &L.ncells);
  if (st != RLB_OK) return st;
  const bool d2 = opt->lattice == RLB_D2Q9;
  if (d2) {
    for (int i = 0; i < n; ++i)
      if (m[i].nz != 1) return RLB_E_ARG;
    if (opt->ckpt_every > 0) return RLB_E_UNSUPPORTED;  // the adjoint covers D3Q19
  }
  if (opt->ckpt_every > 0 && n != 1) return RLB_E_UNSUPPORTED;
  if (opt->ckpt_every > 0 && (m[0].eta_over_s > 0.0 || !paper_eos(m[0])))
    return RLB_E_UNSUPPORTED;  // the adjoint covers fixed taus and P = eps/3
  if (opt->correction)
    for (int i = 0; i < n; ++i)
      if (!paper_eos(m[i])) return RLB_E_UNSUPPORTED;  // C_7 is derived for P = eps/3
  L.esz = opt->precision == RLB_FP32 ? 4 : 8;
  // Plane stride: a multiple of 64 elements plus 1280 bytes, so that planes of
  // a power-of-two lattice do not all start alike on the HBM channels
  // (measured: 3-5 % faster at 256^3 than unpadded planes in both precisions,
  // and at 512^3 FP32 2 % faster than a 256-byte pad).
  L.cs = (L.ncells + 63) / 64 * 64 + kPlanePadBytes / (int64_t)L.esz;
  // every population byte offset of a plane is a 32-bit quantity in the kernels
  if ((uint64_t)L.cs * L.esz >= (uint64_t(1) << 32)) return RLB_E_UNSUPPORTED;
  int parts = std::max<int64_t>(n, (L.ncells + 255) / 256 > 65536 ? 65536 : (L.ncells + 255) / 256);
  if (lattice_path(n, L.ncells)) {
    LatticeGeom g{};
    g.nx = m[0].nx;
    g.ny = m[0].ny;
    g.nz = m[0].nz;
    if (d2) {
      for (int v = 0; v < rlb::d2q9_num_lattice_variants(); ++v)
        parts = std::max(parts, rlb::d2q9_lattice_partials(v, g));
      for (int v = 0; v < rlb::d2q9_num_tile_variants(); ++v) {
        rlb::TileRound a{};
        dim3 grid;
        if (tile_geometry(rlb::d2q9_tile_variant(v), g.nx, g.ny, opt->correction != 0, a, grid))
          parts = std::max<int64_t>(parts, (int64_t)grid.x * grid.y);
      }
    }
    else
      for (int v = 0; v < rlb::num_lattice_variants(); ++v)
        parts = std::max(parts, rlb::lattice_partials(v, g));
  }
  parts = std::max<int64_t>(parts, (int64_t)n * rlb::kRefBlocks);
  if (!lattice_path(n, L.ncells)) {  // segment tables of the persistent path
    // D3Q19: segments of whole z-planes (at most nz per member); D2Q9 strip
    // rounds: segments of whole rows (at most ny per member)
    for (int i = 0; i < n; ++i) L.max_segs += d2 ? m[i].ny : m[i].nz;
    parts = std::max<int64_t>(parts, L.max_segs);
  }
  L.max_parts = std::max(parts, 1);
  size_t o = 0;
  L.off_descs = o;
  o = align_up(o + sizeof(MemberDesc) * n);
  L.off_small = o;
  o = align_up(o + 1024);
  L.off_bad = o;  // the inadmissible-cell slots and their copy kept across tuning trials
  o = align_up(o + 2 * rlb::kBadBytes);
  L.off_partials = o;
  o = align_up(o + sizeof(double) * 5 * (size_t)L.max_parts);
  // The field export keeps its partial sums apart, so that rlb_moments never
  // overwrites the diagnostics partials of the latest step.
  L.export_parts = (int)std::min<int64_t>(std::max<int64_t>((L.ncells + 255) / 256, 1), 65536);
  L.off_xparts = o;
  o = align_up(o + sizeof(double) * 5 * (size_t)L.export_parts);
  const size_t buf = 2 * (size_t)nvel(opt->lattice) * (size_t)L.cs * L.esz;
  L.off_buf0 = o;
  o = align_up(o + buf);
  L.off_buf1 = o;
  o = align_up(o + buf);
  L.off_stage = o;
  o = align_up(o + sizeof(double) * 8 * (size_t)L.ncells);
  L.off_segs = o;
  o = align_up(o + std::max(sizeof(rlb::Segment), sizeof(rlb::TubeSeg)) * (size_t)L.max_segs);
  L.off_flags = o;
  o = align_up(o + sizeof(unsigned long long) * (size_t)L.max_segs);
  L.off_tape = o;
  if (opt->ckpt_every > 0) {
    L.tape = rlb::tape_layout(m[0].nx, m[0].ny, m[0].nz, L.cs, L.esz, opt->ckpt_every,
                              opt->tape_steps, L.max_parts);
    o = align_up(o + L.tape.total);
  }
  L.total = o;
  return RLB_OK;
}

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
      ok = false;
      return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

struct rlb_sim {
  int device = 0;
  hipStream_t stream = nullptr;
  int precision = RLB_FP32;
  rlb_options opt{};
  int n_members = 0;
  std::vector<rlb_params> params;
  std::vector<MemberDesc> descs;  // host copy, refs filled at init
  Layout L;
  char* ws = nullptr;
  MemberDesc* d_descs = nullptr;
  double* d_small = nullptr;  // [0..4] sums out, [8..] scratch
  unsigned long long* d_bad = nullptr;
  unsigned long long* d_count = nullptr;
  unsigned long long* d_bad_total = nullptr;  // the slots' total for the host
  unsigned long long* d_bad_save = nullptr;
  double* d_partials = nullptr;
  double* d_xparts = nullptr;  // export partials (rlb_moments)
  void* buf[2] = {nullptr, nullptr};
  double* d_stage = nullptr;
  int cur = 0;
  bool d2 = false;  // D2Q9 model (9 velocities, 18 planes per buffer)
  bool corr = false;  // D2Q9 with the correction term of Eqs. (37)-(38)
  bool ext = false;    // some member takes its relaxation times from eta/s per cell or
                       // has the general equation of state (the EXT kernels)
  int q = 19;
  bool lattice = false;
  LatticeGeom geom{};
  int variant = 0;
  int64_t steps = 0;
  int64_t diag_step = -1;
  int diag_parts = 0;
  // persistent kernels and their graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraphNode_t gnode = nullptr;
  const void* graph_func = nullptr;
  rlb::MemberLaunch margs{};
  rlb::SegLaunch sargs{};
  rlb::Segment* d_segs = nullptr;
  unsigned long long* d_flags = nullptr;
  int* d_error = nullptr;
  unsigned long long epoch = 0;  // steps every segment flag holds
  int seg_built = -1;             // variant the device segment table describes (segments:
                                  // sv; tube rounds: 1000 + tv; strip rounds: 2000 + sv)
  hipGraph_t tgraph = nullptr;    // chain of tube (or strip) rounds of the last rlb_step
  hipGraphExec_t tgexec = nullptr;
  bool all_tubes = false;
  int nseg = 0;
  int num_cu = 0;
  // tape
  rlb::Tape tape{};
  bool tape_ok = false;
};

namespace {

rlb_status dev_err(hipError_t e) { return e == hipSuccess ? RLB_OK : RLB_E_DEVICE; }

#define RLB_HIP(call)                              \
  do {                                             \
    hipError_t _e = (call);                        \
    if (_e != hipSuccess) return RLB_E_DEVICE;     \
  } while (0)

void* state_buf(rlb_sim* h) { return h->buf[h->cur]; }
void* spare_buf(rlb_sim* h) { return h->buf[1 - h->cur]; }

// Total of the inadmissible-cell slots (count_bad), summed on the device and
// copied back; total() is valid once the stream has reached the copy.
struct BadSlots {
  unsigned long long v = 0;
  hipError_t fetch(const rlb_sim* h) {
    hipError_t e = rlb::launch_sum_bad(h->d_bad, h->d_bad_total, h->stream);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(&v, h->d_bad_total, sizeof(v), hipMemcpyDeviceToHost, h->stream);
  }
  unsigned long long total() const { return v; }
};

rlb_status launch_lattice_step(rlb_sim* h, int variant, bool diag, const void* src, void* dst) {
  if (h->d2)
    return dev_err(rlb::d2q9_launch_step_lattice(h->precision, variant, diag, h->corr, h->ext,
                                                 src, dst, h->geom, h->d_partials, h->d_bad,
                                                 h->stream));
  return dev_err(rlb::launch_step_lattice(h->precision, variant, diag, h->ext, src, dst, h->geom,
                                          h->d_partials, h->d_bad, h->stream));
}

bool is_tile_variant(const rlb_sim* h, int v) {
  return h->lattice && h->d2 && v >= rlb::d2q9_num_lattice_variants();
}

int tile_index(int v) { return v - rlb::d2q9_num_lattice_variants(); }

int lattice_parts(const rlb_sim* h, int variant) {
  if (is_tile_variant(h, variant)) {
    rlb::TileRound a{};
    dim3 grid;
    tile_geometry(rlb::d2q9_tile_variant(tile_index(variant)), h->geom.nx, h->geom.ny, h->corr,
                  a, grid);
    return (int)(grid.x * grid.y);
  }
  return h->d2 ? rlb::d2q9_lattice_partials(variant, h->geom)
               : rlb::lattice_partials(variant, h->geom);
}

// D2Q9 tile rounds: ceil(n / H) launches, each advancing up to H steps of the
// whole lattice; rounds alternate the buffers (pingpong) or always read a and
// write b (trials). *flip tells whether the state changed buffers.
rlb_status launch_tile_rounds(rlb_sim* h, int variant, int nsteps, int pingpong, void* a, void* b,
                              int diag_every, int64_t step0, bool* flip) {
  const rlb::TileVariant v = rlb::d2q9_tile_variant(tile_index(variant));
  rlb::TileRound arg{};
  dim3 grid;
  if (!rlb::d2q9_tile_fits(h->precision, tile_index(variant), h->corr) ||
      !tile_geometry(v, h->geom.nx, h->geom.ny, h->corr, arg, grid))
    return RLB_E_UNSUPPORTED;
  arg.cs = h->L.cs;
  arg.nx = h->geom.nx;
  arg.ny = h->geom.ny;
  arg.bcx = h->geom.bcx;
  arg.bcy = h->geom.bcy;
  arg.diag_every = diag_every;
  arg.last_step = step0 + nsteps;
  arg.rt = h->geom.rt;
  arg.ref = h->geom.ref;
  arg.ext = h->geom.ext;
  arg.partials = h->d_partials;
  arg.bad = h->d_bad;
  const int rounds = (nsteps + v.h - 1) / v.h;
  for (int r = 0; r < rounds; ++r) {
    const bool odd = pingpong && (r & 1);
    arg.src = odd ? b : a;
    arg.dst = odd ? a : b;
    arg.nsteps = std::min(v.h, nsteps - r * v.h);
    arg.step0 = step0 + (int64_t)r * v.h;
    RLB_HIP(rlb::d2q9_launch_tiles(h->precision, tile_index(variant), h->corr, h->ext, arg, grid,
                                   h->stream));
  }
  *flip = pingpong && (rounds & 1);
  return RLB_OK;
}

constexpr int kSpinLimit = 1 << 24;  // about a second of polling per wait

bool is_segment_variant(const rlb_sim* h, int v) {
  return !h->lattice && !h->d2 && v >= rlb::num_member_variants() &&
         v < rlb::num_member_variants() + rlb::num_segment_variants();
}

bool is_tube_variant(const rlb_sim* h, int v) {
  return !h->lattice && !h->d2 &&
         v >= rlb::num_member_variants() + rlb::num_segment_variants();
}

int tube_index(int v) { return v - rlb::num_member_variants() - rlb::num_segment_variants(); }

bool is_strip_variant(const rlb_sim* h, int v) {
  return !h->lattice && h->d2 && v >= rlb::d2q9_num_member_variants();
}

int strip_index(int v) { return v - rlb::d2q9_num_member_variants(); }

// Tube segments for a tube variant: owned ranges of at most NT - 2H cells,
// windows extended by H halo cells (cut at zero-gradient ends); a tube that
// fits the block whole is one segment with exact ends.
rlb_status build_tube_segments(rlb_sim* h, int tv) {
  const rlb::TubeVariant v = rlb::tube_variant(tv);
  const int S = v.nt - 2 * v.halo;
  std::vector<rlb::TubeSeg> segs;
  for (int m = 0; m < h->n_members; ++m) {
    const MemberDesc& d = h->descs[m];
    const int L = d.nz;
    const bool periodic = d.bcz == RLB_PERIODIC;
    if (L <= v.nt) {
      const int kind = periodic ? rlb::kEdgeWrap : rlb::kEdgeClamp;
      segs.push_back(rlb::TubeSeg{m, 0, L, 0, L, kind, kind});
      continue;
    }
    const int n = (L + S - 1) / S;
    for (int j = 0; j < n; ++j) {
      rlb::TubeSeg g{};
      g.member = m;
      g.own0 = (int)((int64_t)L * j / n);
      g.own1 = (int)((int64_t)L * (j + 1) / n);
      if (periodic) {
        g.win0 = g.own0 - v.halo;
        g.wlen = g.own1 - g.own0 + 2 * v.halo;
        g.left = g.right = rlb::kEdgeHalo;
      } else {
        g.win0 = std::max(0, g.own0 - v.halo);
        const int win1 = std::min(L, g.own1 + v.halo);
        g.wlen = win1 - g.win0;
        g.left = g.win0 == 0 ? rlb::kEdgeClamp : rlb::kEdgeHalo;
        g.right = win1 == L ? rlb::kEdgeClamp : rlb::kEdgeHalo;
      }
      segs.push_back(g);
    }
  }
  if ((int64_t)segs.size() > h->L.max_segs) return RLB_E_ARG;
  RLB_HIP(hipMemcpyAsync(h->d_segs, segs.data(), sizeof(rlb::TubeSeg) * segs.size(),
                         hipMemcpyHostToDevice, h->stream));
  RLB_HIP(hipStreamSynchronize(h->stream));
  h->nseg = (int)segs.size();
  h->seg_built = 1000 + tv;
  return RLB_OK;
}

// D2Q9 strip segments for a strip variant: windows of R = nt / nx rows, H
// halo rows a side (2H with the correction term), owned ranges of at most
// R - 2H rows; a member of at most R rows is one segment with exact ends.
// RLB_E_UNSUPPORTED when a member is wider than the block or leaves no
// owned row.
rlb_status build_strip_segments(rlb_sim* h, int sv) {
  const rlb::TubeVariant v = rlb::d2q9_strip_variant(sv);
  const int hr = h->corr ? 2 * v.halo : v.halo;
  std::vector<rlb::TubeSeg> segs;
  for (int m = 0; m < h->n_members; ++m) {
    const MemberDesc& d = h->descs[m];
    if (d.nx > v.nt) return RLB_E_UNSUPPORTED;
    const int R = v.nt / d.nx;
    const int L = d.ny;
    const bool periodic = d.bcy == RLB_PERIODIC;
    if (L <= R) {
      const int kind = periodic ? rlb::kEdgeWrap : rlb::kEdgeClamp;
      segs.push_back(rlb::TubeSeg{m, 0, L, 0, L, kind, kind});
      continue;
    }
    const int S = R - 2 * hr;
    if (S < 1) return RLB_E_UNSUPPORTED;
    const int n = (L + S - 1) / S;
    for (int j = 0; j < n; ++j) {
      rlb::TubeSeg g{};
      g.member = m;
      g.own0 = (int)((int64_t)L * j / n);
      g.own1 = (int)((int64_t)L * (j + 1) / n);
      if (periodic) {
        g.win0 = g.own0 - hr;
        g.wlen = g.own1 - g.own0 + 2 * hr;
        g.left = g.right = rlb::kEdgeHalo;
      } else {
        g.win0 = std::max(0, g.own0 - hr);
        const int win1 = std::min(L, g.own1 + hr);
        g.wlen = win1 - g.win0;
        g.left = g.win0 == 0 ? rlb::kEdgeClamp : rlb::kEdgeHalo;
        g.right = win1 == L ? rlb::kEdgeClamp : rlb::kEdgeHalo;
      }
      segs.push_back(g);
    }
  }
  if ((int64_t)segs.size() > h->L.max_segs) return RLB_E_ARG;
  RLB_HIP(hipMemcpyAsync(h->d_segs, segs.data(), sizeof(rlb::TubeSeg) * segs.size(),
                         hipMemcpyHostToDevice, h->stream));
  RLB_HIP(hipStreamSynchronize(h->stream));
  h->nseg = (int)segs.size();
  h->seg_built = 2000 + sv;
  return RLB_OK;
}

// Tube rounds: ceil(n / H) launches chained in a HIP graph, each round
// reading one buffer and writing the other (pingpong) or always A -> B
// (trials). *flip tells whether the state changed buffers.
// (The D2Q9 strip rounds take the same path with their own segments and
// kernel.)
rlb_status launch_tubes(rlb_sim* h, int variant, int nsteps, int pingpong, void* a, void* b,
                        int diag_every, int64_t step0, bool* flip) {
  rlb::TubeVariant v;
  const void* func;
  dim3 block;
  if (h->d2) {
    const int sv = strip_index(variant);
    if (h->seg_built != 2000 + sv) {
      rlb_status st = build_strip_segments(h, sv);
      if (st != RLB_OK) return st;
    }
    v = rlb::d2q9_strip_variant(sv);
    RLB_HIP(rlb::d2q9_strip_kernel(h->precision, sv, h->corr, h->ext, &func, &block));
  } else {
    const int tv = tube_index(variant);
    if (!h->all_tubes) return RLB_E_UNSUPPORTED;
    if (h->seg_built != 1000 + tv) {
      rlb_status st = build_tube_segments(h, tv);
      if (st != RLB_OK) return st;
    }
    v = rlb::tube_variant(tv);
    RLB_HIP(rlb::tube_kernel(h->precision, tv, h->ext, &func, &block));
  }
  const int rounds = (nsteps + v.halo - 1) / v.halo;
  if (h->tgexec) {  // the previous chain may still run: let it finish first
    RLB_HIP(hipStreamSynchronize(h->stream));
    (void)hipGraphExecDestroy(h->tgexec);
    (void)hipGraphDestroy(h->tgraph);
    h->tgexec = nullptr;
    h->tgraph = nullptr;
  }
  RLB_HIP(hipGraphCreate(&h->tgraph, 0));
  hipGraphNode_t prev = nullptr;
  for (int r = 0; r < rounds; ++r) {
    rlb::TubeRound arg{};
    const bool odd = pingpong && (r & 1);
    arg.descs = h->d_descs;
    arg.segs = (const rlb::TubeSeg*)h->d_segs;
    arg.src = odd ? b : a;
    arg.dst = odd ? a : b;
    arg.cs = h->L.cs;
    arg.nsteps = std::min(v.halo, nsteps - r * v.halo);
    arg.diag_every = diag_every;
    arg.step0 = step0 + (int64_t)r * v.halo;
    arg.last_step = step0 + nsteps;
    arg.partials = h->d_partials;
    arg.bad = h->d_bad;
    void* args[] = {&arg};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(func);
    kp.gridDim = dim3(h->nseg, 1, 1);
    kp.blockDim = block;
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    RLB_HIP(hipGraphAddKernelNode(&node, h->tgraph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
    prev = node;
  }
  RLB_HIP(hipGraphInstantiate(&h->tgexec, h->tgraph, nullptr, nullptr, 0));
  RLB_HIP(hipGraphLaunch(h->tgexec, h->stream));
  *flip = pingpong && (rounds & 1);
  return RLB_OK;
}

// Cut every member into segments of whole z-planes of about nt * cpt cells
// (one pass of the block per step) and upload the table.
rlb_status build_segments(rlb_sim* h, int sv) {
  const rlb::MemberVariant mv = rlb::segment_variant(sv);
  const int64_t target = (int64_t)mv.nt * mv.cpt;
  std::vector<rlb::Segment> segs;
  for (int m = 0; m < h->n_members; ++m) {
    const MemberDesc& d = h->descs[m];
    const int64_t plane = (int64_t)d.nx * d.ny;
    const int64_t want = std::max<int64_t>(1, (d.ncells + target - 1) / target);
    const int nsm = (int)std::min<int64_t>(want, d.nz);
    const int first = (int)segs.size();
    for (int j = 0; j < nsm; ++j) {
      rlb::Segment g{};
      g.member = m;
      g.z0 = (int)((int64_t)d.nz * j / nsm);
      g.z1 = (int)((int64_t)d.nz * (j + 1) / nsm);
      const bool wrap = d.bcz == RLB_PERIODIC && nsm > 1;
      g.left = j > 0 ? first + j - 1 : (wrap ? first + nsm - 1 : -1);
      g.right = j < nsm - 1 ? first + j + 1 : (wrap ? first : -1);
      segs.push_back(g);
      (void)plane;
    }
  }
  if ((int64_t)segs.size() > h->L.max_segs) return RLB_E_ARG;
  RLB_HIP(hipMemcpyAsync(h->d_segs, segs.data(), sizeof(rlb::Segment) * segs.size(),
                         hipMemcpyHostToDevice, h->stream));
  RLB_HIP(hipStreamSynchronize(h->stream));
  h->nseg = (int)segs.size();
  h->seg_built = sv;
  return RLB_OK;
}

// Every block of a segment launch must be resident at once (they wait on
// each other); variants whose segments do not fit are refused.
rlb_status segments_fit(rlb_sim* h, int sv, const void* func, int nt) {
  if (h->seg_built != sv) {
    rlb_status st = build_segments(h, sv);
    if (st != RLB_OK) return st;
  }
  int per_cu = 0;
  RLB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, func, nt, 0));
  if ((int64_t)per_cu * h->num_cu < h->nseg) return RLB_E_UNSUPPORTED;
  return RLB_OK;
}

// Persistent kernels run from a one-node HIP graph (built on first use, and
// again when the kernel changes; later calls only update the arguments).
rlb_status launch_persistent(rlb_sim* h, int variant, int nsteps, int pingpong, void* a, void* b,
                             int diag_every, int64_t step0, bool* flip) {
  if (is_tube_variant(h, variant) || is_strip_variant(h, variant))
    return launch_tubes(h, variant, nsteps, pingpong, a, b, diag_every, step0, flip);
  *flip = pingpong && (nsteps & 1);
  const void* func;
  dim3 block, grid;
  void* args[1];
  if (is_segment_variant(h, variant)) {
    if (h->ext) return RLB_E_UNSUPPORTED;  // fixed relaxation times only
    const int sv = variant - rlb::num_member_variants();
    RLB_HIP(rlb::segment_kernel(h->precision, sv, &func, &block));
    rlb_status st = segments_fit(h, sv, func, block.x);
    if (st != RLB_OK) return st;
    rlb::SegLaunch& g = h->sargs;
    g.descs = h->d_descs;
    g.segs = h->d_segs;
    g.bufA = a;
    g.bufB = b;
    g.cs = h->L.cs;
    g.nsteps = nsteps;
    g.pingpong = pingpong;
    g.diag_every = diag_every;
    g.spin_limit = kSpinLimit;
    g.step0 = step0;
    g.epoch = h->epoch;
    g.flags = h->d_flags;
    g.error = h->d_error;
    g.partials = h->d_partials;
    g.bad = h->d_bad;
    args[0] = &h->sargs;
    grid = dim3(h->nseg, 1, 1);
  } else {
    rlb::MemberLaunch& m = h->margs;
    m.descs = h->d_descs;
    m.bufA = a;
    m.bufB = b;
    m.cs = h->L.cs;
    m.nsteps = nsteps;
    m.pingpong = pingpong;
    m.diag_every = diag_every;
    m.step0 = step0;
    m.partials = h->d_partials;
    m.bad = h->d_bad;
    if (h->d2)
      RLB_HIP(rlb::d2q9_member_kernel(h->precision, variant, h->corr, h->ext, &func, &block));
    else
      RLB_HIP(rlb::member_kernel(h->precision, variant, h->ext, &func, &block));
    args[0] = &h->margs;
    grid = dim3(h->n_members, 1, 1);
  }
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(func);
  kp.gridDim = grid;
  kp.blockDim = block;
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  if (h->gexec && h->graph_func != func) {
    RLB_HIP(hipStreamSynchronize(h->stream));
    (void)hipGraphExecDestroy(h->gexec);
    (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
  }
  if (!h->gexec) {
    RLB_HIP(hipGraphCreate(&h->graph, 0));
    RLB_HIP(hipGraphAddKernelNode(&h->gnode, h->graph, nullptr, 0, &kp));
    RLB_HIP(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
    h->graph_func = func;
  } else {
    RLB_HIP(hipGraphExecKernelNodeSetParams(h->gexec, h->gnode, &kp));
  }
  RLB_HIP(hipGraphLaunch(h->gexec, h->stream));
  if (is_segment_variant(h, variant)) h->epoch += (unsigned long long)nsteps;
  return RLB_OK;
}

// Advance n steps without taping.
rlb_status advance(rlb_sim* h, int32_t n) {
  if (n <= 0) return RLB_OK;
  const int D = h->opt.diag_every;
  if (h->lattice && is_tile_variant(h, h->variant)) {
    bool flip = false;
    rlb_status st =
        launch_tile_rounds(h, h->variant, n, 1, state_buf(h), spare_buf(h), D, h->steps, &flip);
    if (st != RLB_OK) return st;
    if (D > 0) {
      h->diag_step = h->steps + n;
      h->diag_parts = lattice_parts(h, h->variant);
    }
    h->steps += n;
    if (flip) h->cur = 1 - h->cur;
    return RLB_OK;
  }
  if (h->lattice) {
    for (int32_t i = 0; i < n; ++i) {
      const int64_t s = h->steps + 1;
      const bool diag = D > 0 && (s % D == 0 || i == n - 1);
      rlb_status st = launch_lattice_step(h, h->variant, diag, state_buf(h), spare_buf(h));
      if (st != RLB_OK) return st;
      if (diag) {
        h->diag_step = s;
        h->diag_parts = lattice_parts(h, h->variant);
      }
      h->cur = 1 - h->cur;
      h->steps = s;
    }
    return RLB_OK;
  }
  bool flip = false;
  rlb_status st =
      launch_persistent(h, h->variant, n, 1, state_buf(h), spare_buf(h), D, h->steps, &flip);
  if (st != RLB_OK) return st;
  if (D > 0) {
    h->diag_step = h->steps + n;
    const bool by_seg = is_segment_variant(h, h->variant) || is_tube_variant(h, h->variant) ||
                        is_strip_variant(h, h->variant);
    h->diag_parts = by_seg ? h->nseg : h->n_members;
  }
  h->steps += n;
  if (flip) h->cur = 1 - h->cur;
  return RLB_OK;
}

rlb_status copy_fields_in(rlb_sim* h, const double* n0, const double* eps0, const double* u0,
                          int on_device, const double** dn, const double** de,
                          const double** du) {
  const int64_t nc = h->L.ncells;
  if (on_device) {
    *dn = n0;
    *de = eps0;
    *du = u0;
    return RLB_OK;
  }
  double* s = h->d_stage;
  RLB_HIP(hipMemcpyAsync(s, n0, sizeof(double) * nc, hipMemcpyHostToDevice, h->stream));
  RLB_HIP(hipMemcpyAsync(s + nc, eps0, sizeof(double) * nc, hipMemcpyHostToDevice, h->stream));
  RLB_HIP(
      hipMemcpyAsync(s + 2 * nc, u0, sizeof(double) * 3 * nc, hipMemcpyHostToDevice, h->stream));
  *dn = s;
  *de = s + nc;
  *du = s + 2 * nc;
  return RLB_OK;
}

bool host_fields_ok(const double* n0, const double* eps0, const double* u0, int64_t nc,
                    bool planar, const rlb_params* members, int32_t n_members) {
  int64_t i = 0;
  for (int m = 0; m < n_members; ++m) {
    const rlb_params& p = members[m];
    const int64_t end = i + (int64_t)p.nx * p.ny * p.nz;
    const bool gen = !paper_eos(p);
    for (; i < end; ++i) {
      const double uu =
          u0[i] * u0[i] + u0[nc + i] * u0[nc + i] + u0[2 * nc + i] * u0[2 * nc + i];
      if (!(eps0[i] > 0.0) || !(n0[i] >= 0.0) || !(uu < 1.0) || !std::isfinite(n0[i]) ||
          !std::isfinite(eps0[i]) || (planar && u0[2 * nc + i] != 0.0) ||
          (gen && !(eps0[i] - p.mass * n0[i] > 0.0)))
        return false;
    }
  }
  return true;
}

}  // namespace

namespace {

const char* kernel_name_of(const rlb_sim* h, int v) {
  if (h->d2) {
    if (is_tile_variant(h, v)) return rlb::d2q9_tile_kernel_name(h->precision, tile_index(v));
    if (h->lattice) return rlb::d2q9_lattice_kernel_name(h->precision, v);
    if (is_strip_variant(h, v)) return rlb::d2q9_strip_kernel_name(h->precision, strip_index(v));
    return rlb::d2q9_member_kernel_name(h->precision, v);
  }
  if (h->lattice) return rlb::lattice_kernel_name(h->precision, v);
  if (v < rlb::num_member_variants()) return rlb::member_kernel_name(h->precision, v);
  if (is_segment_variant(h, v))
    return rlb::segment_kernel_name(h->precision, v - rlb::num_member_variants());
  return rlb::tube_kernel_name(h->precision, tube_index(v));
}

// A persistent segment launch whose neighbour wait timed out leaves a sticky
// error word; it is reported at the next synchronising call.
rlb_status persistent_error(rlb_sim* h) {
  int e = 0;
  RLB_HIP(hipMemcpyAsync(&e, h->d_error, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  RLB_HIP(hipStreamSynchronize(h->stream));
  return e ? RLB_E_DEVICE : RLB_OK;
}

}  // namespace

// ============================================================================
extern "C" {

static_assert(sizeof(rlb_status) == sizeof(int32_t), "rlb_status travels as a 32-bit int");

const char* rlb_status_string(rlb_status s) {
  // A C caller may pass any int: read it as one (loading an enum object that
  // holds a value outside the enumeration's range is undefined in C++).
  int32_t code;
  std::memcpy(&code, &s, sizeof(code));
  switch (code) {
    case RLB_OK: return "ok";
    case RLB_E_ARG: return "invalid argument";
    case RLB_E_TAU: return "relaxation time must be finite and > 1/2";
    case RLB_E_UNPHYSICAL: return "inadmissible cell (eps <= 0, n < 0, |u| >= 1 or E <= 0, |M| >= E)";
    case RLB_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case RLB_E_DEVICE: return "HIP runtime error";
    case RLB_E_STATE: return "call not valid in the current state";
    case RLB_E_UNSUPPORTED: return "unsupported configuration";
    case RLB_E_SCRATCH: return "lattice too large for the fixed scratch array of rlb_run_noalloc";
  }
  return "unknown status";
}

rlb_status rlb_workspace_size(const rlb_params* members, int32_t n_members,
                              const rlb_options* opt, size_t* bytes) {
  if (!bytes) return RLB_E_ARG;
  Layout L;
  rlb_status st = make_layout(members, n_members, opt, L);
  if (st != RLB_OK) return st;
  *bytes = L.total;
  return RLB_OK;
}

rlb_status rlb_init(rlb_handle* out, const rlb_params* members, int32_t n_members,
                    const rlb_options* opt, const double* n0, const double* eps0,
                    const double* u0, int32_t fields_on_device, void* workspace,
                    size_t workspace_bytes, void* hip_stream) {
  if (!out) return RLB_E_ARG;
  *out = nullptr;
  Layout L;
  rlb_status st = make_layout(members, n_members, opt, L);
  if (st != RLB_OK) return st;
  if (!n0 || !eps0 || !u0) return RLB_E_ARG;
  if (fields_on_device != 0 && fields_on_device != 1) return RLB_E_ARG;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || workspace_bytes < L.total)
    return RLB_E_WORKSPACE;
  const bool planar = opt->lattice == RLB_D2Q9;
  if (!fields_on_device && !host_fields_ok(n0, eps0, u0, L.ncells, planar, members, n_members))
    return RLB_E_UNPHYSICAL;

  rlb_sim* h = new (std::nothrow) rlb_sim();
  if (!h) return RLB_E_ARG;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return RLB_E_DEVICE;
  }
  h->stream = (hipStream_t)hip_stream;
  h->precision = opt->precision;
  h->opt = *opt;
  h->n_members = n_members;
  h->params.assign(members, members + n_members);
  h->L = L;
  h->ws = (char*)workspace;
  h->d_descs = (MemberDesc*)(h->ws + L.off_descs);
  h->d_small = (double*)(h->ws + L.off_small);
  h->d_count = (unsigned long long*)(h->d_small + 16);
  h->d_bad_total = (unsigned long long*)(h->d_small + 20);
  h->d_bad = (unsigned long long*)(h->ws + L.off_bad);
  h->d_bad_save = h->d_bad + rlb::kBadBytes / sizeof(unsigned long long);
  h->d_partials = (double*)(h->ws + L.off_partials);
  h->d_xparts = (double*)(h->ws + L.off_xparts);
  h->buf[0] = h->ws + L.off_buf0;
  h->buf[1] = h->ws + L.off_buf1;
  h->d_stage = (double*)(h->ws + L.off_stage);
  h->d_segs = (rlb::Segment*)(h->ws + L.off_segs);
  h->d_flags = (unsigned long long*)(h->ws + L.off_flags);
  h->d_error = (int*)(h->d_small + 24);
  h->d2 = planar;
  h->corr = opt->correction != 0;
  h->q = nvel(opt->lattice);
  h->lattice = lattice_path(n_members, L.ncells);
  // defaults: the lattice path's 256 x 1 block; the persistent path's 512
  // threads with one cell each
  h->variant = h->d2 ? (h->lattice ? 2 : 1) : (h->lattice ? 3 : 1);
  h->all_tubes = !h->d2;
  for (int i = 0; i < n_members; ++i)
    if (members[i].nx != 1 || members[i].ny != 1) h->all_tubes = false;

  auto fail = [&](rlb_status s) {
    delete h;
    return s;
  };
  // member descriptors (refs are filled on the device)
  h->descs.resize(n_members);
  int64_t off = 0;
  for (int i = 0; i < n_members; ++i) {
    const rlb_params& p = members[i];
    MemberDesc& d = h->descs[i];
    std::memset(&d, 0, sizeof(d));
    d.offset = off;
    d.nx = p.nx;
    d.ny = p.ny;
    d.nz = p.nz;
    d.ncells = p.nx * p.ny * p.nz;
    d.bcx = p.bc[0];
    d.bcy = p.bc[1];
    d.bcz = p.bc[2];
    const double tq = p.tau_q > 0.0 ? p.tau_q : p.tau_v;
    d.rt.w_f = 1.0 / p.tau_f;
    d.rt.s_e = 1.0 / p.tau_e;
    d.rt.s_eps = 1.0 / p.tau_eps;
    d.rt.s_q = 1.0 / tq;
    d.rt.s_v = 1.0 / p.tau_v;
    d.ext.eta_s = p.eta_over_s;
    d.ext.kappa = p.kappa;
    d.ext.dof = p.dof;
    d.ext.a_f = p.a_f;
    d.ext.a_e = p.a_e;
    d.ext.a_eps = p.a_eps;
    d.ext.a_q = p.a_q;
    d.ext.q_tied = p.tau_q > 0.0 ? 0 : 1;
    d.ext.eos_gamma = p.eos_gamma > 0.0 ? p.eos_gamma : 4.0 / 3.0;
    d.ext.mass = p.mass;
    d.ext.general_eos = paper_eos(p) ? 0 : 1;
    if (p.eta_over_s > 0.0 || d.ext.general_eos) h->ext = true;
    off += d.ncells;
  }
  const double *dn, *de, *du;
  if (hipMemsetAsync(h->d_small, 0, 1024, h->stream) != hipSuccess ||
      hipMemsetAsync(h->d_bad, 0, rlb::kBadBytes, h->stream) != hipSuccess)
    return fail(RLB_E_DEVICE);
  if (L.max_segs > 0 &&
      hipMemsetAsync(h->d_flags, 0, sizeof(unsigned long long) * L.max_segs, h->stream) !=
          hipSuccess)
    return fail(RLB_E_DEVICE);
  if (hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, h->device) !=
      hipSuccess)
    return fail(RLB_E_DEVICE);
  if (copy_fields_in(h, n0, eps0, u0, fields_on_device, &dn, &de, &du) != RLB_OK)
    return fail(RLB_E_DEVICE);
  if (hipMemcpyAsync(h->d_descs, h->descs.data(), sizeof(MemberDesc) * n_members,
                     hipMemcpyHostToDevice, h->stream) != hipSuccess)
    return fail(RLB_E_DEVICE);
  if (fields_on_device) {
    if (rlb::launch_validate(dn, de, du, L.ncells, planar ? 1 : 0, h->d_descs, n_members,
                             h->d_count, h->stream) != hipSuccess)
      return fail(RLB_E_DEVICE);
    unsigned long long cnt = 0;
    if (hipMemcpyAsync(&cnt, h->d_count, sizeof(cnt), hipMemcpyDeviceToHost, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
      return fail(RLB_E_DEVICE);
    if (cnt) return fail(RLB_E_UNPHYSICAL);
  }
  if (rlb::launch_member_refs(h->d_descs, n_members, dn, de, du, L.ncells, h->d_partials,
                              h->stream) != hipSuccess)
    return fail(RLB_E_DEVICE);
  const hipError_t ie =
      planar ? rlb::d2q9_launch_init(h->precision, h->buf[0], L.cs, h->d_descs, n_members, dn,
                                     de, du, L.ncells, h->stream)
             : rlb::launch_init(h->precision, h->buf[0], L.cs, h->d_descs, n_members, dn, de, du,
                                L.ncells, h->stream);
  if (ie != hipSuccess) return fail(RLB_E_DEVICE);
  if (hipMemcpyAsync(h->descs.data(), h->d_descs, sizeof(MemberDesc) * n_members,
                     hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return fail(RLB_E_DEVICE);
  if (h->lattice) {
    const MemberDesc& d = h->descs[0];
    h->geom.nx = d.nx;
    h->geom.ny = d.ny;
    h->geom.nz = d.nz;
    h->geom.bcx = d.bcx;
    h->geom.bcy = d.bcy;
    h->geom.bcz = d.bcz;
    h->geom.cs = L.cs;
    h->geom.rt = d.rt;
    h->geom.ref = d.ref;
    h->geom.ext = d.ext;
    // Plain stores in the one-step kernels while the double-buffered state is
    // at most 1 GiB (measured on D3Q19 FP32 planar lattices: 25-37 % faster
    // at 80-160 MB, even at 320 MB, 10 % faster at 640 MB; nontemporal stores
    // 4-5 % faster from 1.3 GB up, e.g. the 5.1 GB of 256^3).
    h->geom.cached_store = 2 * (L.off_buf1 - L.off_buf0) <= kCachedStateBytes ? 1 : 0;
  }
  h->cur = 0;
  if (opt->ckpt_every > 0) {
    rlb_status ts = rlb::tape_init(h->tape, L.tape, h->ws + L.off_tape, h->precision, L.ncells,
                                   L.cs, opt->ckpt_every, opt->tape_steps, dn, de, du,
                                   h->buf[0], h->stream);
    if (ts != RLB_OK) return fail(ts);
    h->tape_ok = true;
  }
  *out = h;
  return RLB_OK;
}

rlb_status rlb_step(rlb_handle h, int32_t nsteps) {
  if (!h || nsteps < 0) return RLB_E_ARG;
  if (nsteps == 0) return RLB_OK;
  DeviceGuard g(h->device);
  if (!g.ok) return RLB_E_DEVICE;
  if (h->opt.ckpt_every <= 0 || !h->tape_ok) return advance(h, nsteps);
  // With a tape: stop at every checkpoint boundary and keep g.
  const int K = h->opt.ckpt_every;
  int32_t left = nsteps;
  while (left > 0) {
    int32_t chunk = (int32_t)std::min<int64_t>(left, K - (h->steps % K));
    rlb_status st = advance(h, chunk);
    if (st != RLB_OK) return st;
    left -= chunk;
    if (h->steps > h->opt.tape_steps) {
      h->tape_ok = false;
      return advance(h, left);
    }
    if (h->steps % K == 0) {
      st = rlb::tape_checkpoint(h->tape, h->steps / K, state_buf(h), h->stream);
      if (st != RLB_OK) return st;
    }
  }
  return RLB_OK;
}

rlb_status rlb_moments(rlb_handle h, double* n, double* eps, double* P, double* gamma,
                       double* u, double sums[5], int64_t* n_unphysical,
                       int32_t out_on_device) {
  if (!h) return RLB_E_ARG;
  if (out_on_device != 0 && out_on_device != 1) return RLB_E_ARG;
  DeviceGuard g(h->device);
  if (!g.ok) return RLB_E_DEVICE;
  const int64_t nc = h->L.ncells;
  double* s = h->d_stage;
  double *dn = n, *de = eps, *dP = P, *dg = gamma, *du = u;
  if (!out_on_device) {
    dn = n ? s : nullptr;
    de = eps ? s + nc : nullptr;
    dP = P ? s + 2 * nc : nullptr;
    dg = gamma ? s + 3 * nc : nullptr;
    du = u ? s + 4 * nc : nullptr;
  }
  const int nparts = h->L.export_parts;
  if (h->d2)
    RLB_HIP(rlb::d2q9_launch_export(h->precision, state_buf(h), h->L.cs, h->d_descs,
                                    h->n_members, nc, dn, de, dP, dg, du, h->d_xparts, nparts,
                                    h->stream));
  else
    RLB_HIP(rlb::launch_export(h->precision, state_buf(h), h->L.cs, h->d_descs, h->n_members,
                               nc, dn, de, dP, dg, du, h->d_xparts, nparts, h->stream));
  RLB_HIP(rlb::launch_reduce(h->d_xparts, nparts, h->d_small, h->stream));
  double hs[5];
  BadSlots slots;
  RLB_HIP(hipMemcpyAsync(hs, h->d_small, sizeof(hs), hipMemcpyDeviceToHost, h->stream));
  RLB_HIP(slots.fetch(h));
  if (!out_on_device) {
    if (n) RLB_HIP(hipMemcpyAsync(n, dn, sizeof(double) * nc, hipMemcpyDeviceToHost, h->stream));
    if (eps)
      RLB_HIP(hipMemcpyAsync(eps, de, sizeof(double) * nc, hipMemcpyDeviceToHost, h->stream));
    if (P) RLB_HIP(hipMemcpyAsync(P, dP, sizeof(double) * nc, hipMemcpyDeviceToHost, h->stream));
    if (gamma)
      RLB_HIP(hipMemcpyAsync(gamma, dg, sizeof(double) * nc, hipMemcpyDeviceToHost, h->stream));
    if (u)
      RLB_HIP(hipMemcpyAsync(u, du, sizeof(double) * 3 * nc, hipMemcpyDeviceToHost, h->stream));
  }
  RLB_HIP(hipStreamSynchronize(h->stream));
  const unsigned long long bad = slots.total();
  if (sums) std::memcpy(sums, hs, sizeof(hs));
  if (n_unphysical) *n_unphysical = (int64_t)bad;
  if (persistent_error(h) != RLB_OK) return RLB_E_DEVICE;
  return bad ? RLB_E_UNPHYSICAL : RLB_OK;
}

rlb_status rlb_diagnostics(rlb_handle h, double sums[5], int64_t* step, int64_t* n_unphysical) {
  if (!h) return RLB_E_ARG;
  if (h->diag_step < 0) return RLB_E_STATE;
  DeviceGuard g(h->device);
  if (!g.ok) return RLB_E_DEVICE;
  RLB_HIP(rlb::launch_reduce(h->d_partials, h->diag_parts, h->d_small, h->stream));
  double hs[5];
  BadSlots slots;
  RLB_HIP(hipMemcpyAsync(hs, h->d_small, sizeof(hs), hipMemcpyDeviceToHost, h->stream));
  RLB_HIP(slots.fetch(h));
  RLB_HIP(hipStreamSynchronize(h->stream));
  if (sums) std::memcpy(sums, hs, sizeof(hs));
  if (step) *step = h->diag_step;
  if (n_unphysical) *n_unphysical = (int64_t)slots.total();
  return persistent_error(h);
}

rlb_status rlb_populations(rlb_handle h, double* f, double* g, int32_t out_on_device) {
  if (!h) return RLB_E_ARG;
  if (out_on_device != 0 && out_on_device != 1) return RLB_E_ARG;
  DeviceGuard dg(h->device);
  if (!dg.ok) return RLB_E_DEVICE;
  const int64_t nc = h->L.ncells;
  const int Q = h->q;
  auto planes = [&](int p0, int np, double* out) {
    return h->d2 ? rlb::d2q9_launch_population_planes(h->precision, state_buf(h), h->L.cs,
                                                      h->d_descs, h->n_members, nc, p0, np, out,
                                                      h->stream)
                 : rlb::launch_population_planes(h->precision, state_buf(h), h->L.cs,
                                                 h->d_descs, h->n_members, nc, p0, np, out,
                                                 h->stream);
  };
  if (out_on_device) {
    if (f) RLB_HIP(planes(0, Q, f));
    if (g) RLB_HIP(planes(Q, Q, g));
  } else {
    // staging holds 8 planes: convert f (then g) in chunks of up to 8 planes
    double* s = h->d_stage;
    for (int which = 0; which < 2; ++which) {
      double* hostp = which ? g : f;
      if (!hostp) continue;
      for (int a0 = 0; a0 < Q; a0 += 8) {
        const int na = std::min(8, Q - a0);
        RLB_HIP(planes(which * Q + a0, na, s));
        RLB_HIP(hipMemcpyAsync(hostp + (size_t)a0 * nc, s, sizeof(double) * na * nc,
                               hipMemcpyDeviceToHost, h->stream));
        RLB_HIP(hipStreamSynchronize(h->stream));
      }
    }
  }
  RLB_HIP(hipStreamSynchronize(h->stream));
  return persistent_error(h);
}

rlb_status rlb_grad(rlb_handle h, const double* dL_du, const double* dL_deps,
                    double dL_dtau[3], double* dL_deps0, double* dL_du0, int32_t io_on_device) {
  if (!h || !dL_du || !dL_deps || !dL_dtau || !dL_deps0 || !dL_du0) return RLB_E_ARG;
  if (io_on_device != 0 && io_on_device != 1) return RLB_E_ARG;
  if (h->opt.ckpt_every <= 0 || !h->tape_ok) return RLB_E_STATE;
  DeviceGuard g(h->device);
  if (!g.ok) return RLB_E_DEVICE;
  rlb::GradContext c{};
  c.precision = h->precision;
  c.ncells = h->L.ncells;
  c.cs = h->L.cs;
  c.desc = h->descs[0];
  c.steps = h->steps;
  c.tau_q_tied = !(h->params[0].tau_q > 0.0);
  c.state = state_buf(h);
  c.stage = h->d_stage;
  c.sums_out = h->d_small;
  c.stream = h->stream;
  return rlb::tape_grad(h->tape, c, dL_du, dL_deps, dL_dtau, dL_deps0, dL_du0, io_on_device);
}

rlb_status rlb_num_variants(rlb_handle h, int32_t* count) {
  if (!h || !count) return RLB_E_ARG;
  if (h->d2)
    *count = h->lattice ? rlb::d2q9_num_lattice_variants() + rlb::d2q9_num_tile_variants()
                        : rlb::d2q9_num_member_variants() + rlb::d2q9_num_strip_variants();
  else
    *count = h->lattice ? rlb::num_lattice_variants()
                        : rlb::num_member_variants() + rlb::num_segment_variants() +
                              rlb::num_tube_variants();
  return RLB_OK;
}

rlb_status rlb_variant_name(rlb_handle h, int32_t v, char* buf, size_t buflen) {
  int32_t n;
  if (rlb_num_variants(h, &n) != RLB_OK || !buf || buflen == 0) return RLB_E_ARG;
  if (v < 0 || v >= n) return RLB_E_ARG;
  std::snprintf(buf, buflen, "%s%s", kernel_name_of(h, v), h->corr ? "+c7" : "");
  return RLB_OK;
}

rlb_status rlb_set_variant(rlb_handle h, int32_t v) {
  int32_t n;
  if (rlb_num_variants(h, &n) != RLB_OK) return RLB_E_ARG;
  if (v < 0 || v >= n) return RLB_E_ARG;
  h->variant = v;
  return RLB_OK;
}

rlb_status rlb_get_variant(rlb_handle h, int32_t* v) {
  if (!h || !v) return RLB_E_ARG;
  *v = h->variant;
  return RLB_OK;
}

rlb_status rlb_tune(rlb_handle h, int32_t trial_steps, int32_t* best_variant,
                    double* ms_per_step) {
  if (!h || trial_steps < 1) return RLB_E_ARG;
  DeviceGuard g(h->device);
  if (!g.ok) return RLB_E_DEVICE;
  int32_t n;
  rlb_num_variants(h, &n);
  hipEvent_t e0, e1;
  RLB_HIP(hipEventCreate(&e0));
  RLB_HIP(hipEventCreate(&e1));
  // trial steps must not count toward the inadmissible-cell total
  RLB_HIP(hipMemcpyAsync(h->d_bad_save, h->d_bad, rlb::kBadBytes, hipMemcpyDeviceToDevice,
                         h->stream));
  const int keep = h->variant;
  int best = keep;
  double best_ms = 1e300;
  rlb_status st = RLB_OK;
  for (int v = 0; v < n && st == RLB_OK; ++v) {
    float ms = 0.0f;
    bool usable = true;
    for (int rep = 0; rep < 2 && st == RLB_OK && usable; ++rep) {  // rep 0 warms up
      if (hipEventRecord(e0, h->stream) != hipSuccess) st = RLB_E_DEVICE;
      if (h->lattice && is_tile_variant(h, v)) {
        bool flip = false;
        st = launch_tile_rounds(h, v, trial_steps, 0, state_buf(h), spare_buf(h), 0, 0, &flip);
        if (st == RLB_E_UNSUPPORTED) {  // a tiled axis leaves no owned cell
          usable = false;
          st = RLB_OK;
        }
      } else if (h->lattice) {
        for (int i = 0; i < trial_steps && st == RLB_OK; ++i)
          st = launch_lattice_step(h, v, false, state_buf(h), spare_buf(h));
      } else if (st == RLB_OK) {
        bool flip = false;
        st = launch_persistent(h, v, trial_steps, 0, state_buf(h), spare_buf(h), 0, 0, &flip);
        if (st == RLB_E_UNSUPPORTED) {  // segments do not all fit at once
          usable = false;
          st = RLB_OK;
        }
      }
      if (st == RLB_OK && usable && hipEventRecord(e1, h->stream) != hipSuccess)
        st = RLB_E_DEVICE;
      if (st == RLB_OK && usable && hipEventSynchronize(e1) != hipSuccess) st = RLB_E_DEVICE;
      if (st == RLB_OK && usable && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        st = RLB_E_DEVICE;
    }
    const double per = usable ? (double)ms / trial_steps : HUGE_VAL;
    if (ms_per_step) ms_per_step[v] = per;
    if (st == RLB_OK && usable && per < best_ms) {
      best_ms = per;
      best = v;
    }
  }
  if (st == RLB_OK) st = persistent_error(h);
  (void)hipMemcpyAsync(h->d_bad, h->d_bad_save, rlb::kBadBytes, hipMemcpyDeviceToDevice,
                       h->stream);
  (void)hipStreamSynchronize(h->stream);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->variant = (st == RLB_OK) ? best : keep;
  if (best_variant) *best_variant = h->variant;
  return st;
}

rlb_status rlb_info(rlb_handle h, int64_t* steps, char* kernel_name, size_t buflen) {
  if (!h) return RLB_E_ARG;
  if (steps) *steps = h->steps;
  if (kernel_name && buflen)
    std::snprintf(kernel_name, buflen, "%s%s", kernel_name_of(h, h->variant),
                  h->corr ? "+c7" : "");
  return RLB_OK;
}

void rlb_free(rlb_handle h) {
  if (!h) return;
  {
    DeviceGuard g(h->device);
    (void)hipStreamSynchronize(h->stream);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->tgexec) (void)hipGraphExecDestroy(h->tgexec);
    if (h->tgraph) (void)hipGraphDestroy(h->tgraph);
    rlb::tape_release(h->tape);
  }
  delete h;
}

}  // extern "C"
