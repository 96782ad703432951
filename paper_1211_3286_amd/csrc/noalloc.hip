// rlb_run_noalloc (include/rlb.h): the run of rlb_init + rlb_step +
// rlb_moments on one lattice, for callers that cannot allocate. Everything the
// kernels need besides the caller's fields (populations, member descriptor,
// partial sums, counters) lives in one fixed device array of this file.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/rlb.h"
#include "internal.hpp"

namespace {

// The fixed scratch array. In host code its name is only a stand-in for the
// device symbol: the device address comes from hipGetSymbolAddress, once per
// device, and only that address is handed to kernels and copies.
static __device__ __align__(256) unsigned char scratch[RLB_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
constexpr size_t kAlign = 256;

struct DeviceSlot {
  std::mutex mu;           // one call at a time per device: the array is shared
  unsigned char* ptr = nullptr;  // device address of this device's copy of scratch
};
DeviceSlot g_slots[kMaxDevices];

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

__global__ void k_zero(unsigned long long* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Carving of the scratch array for one lattice of ncells cells.
struct Carve {
  size_t desc, small, bad, parts, xparts, buf0, buf1, total;
  int64_t cs;
  int export_parts;
};

Carve carve(int64_t ncells, int q, size_t esz) {
  Carve c{};
  c.cs = (ncells + 63) / 64 * 64 + 64;
  c.export_parts = (int)std::min<int64_t>(std::max<int64_t>((ncells + 255) / 256, 1), 65536);
  size_t o = 0;
  c.desc = o;
  o = align_up(o + sizeof(rlb::MemberDesc));
  c.small = o;  // [0..4] sums, [16] validation count, [20] inadmissible total
  o = align_up(o + 1024);
  c.bad = o;
  o = align_up(o + rlb::kBadBytes);
  c.parts = o;
  o = align_up(o + sizeof(double) * 5 * rlb::kRefBlocks);
  c.xparts = o;
  o = align_up(o + sizeof(double) * 5 * (size_t)c.export_parts);
  const size_t buf = 2 * (size_t)q * (size_t)c.cs * esz;
  c.buf0 = o;
  o = align_up(o + buf);
  c.buf1 = o;
  o = align_up(o + buf);
  c.total = o;
  return c;
}

bool paper_eos(const rlb_params& p) {
  return (p.eos_gamma == 0.0 || p.eos_gamma == 4.0 / 3.0) && p.mass == 0.0;
}

bool finite_tau(double t) { return std::isfinite(t) && t > 0.5; }

// The checks rlb_init makes on one member and the options (its make_layout).
rlb_status check(const rlb_params& p, const rlb_options& o) {
  if (o.precision != RLB_FP32 && o.precision != RLB_FP64) return RLB_E_ARG;
  if (o.lattice != RLB_D3Q19 && o.lattice != RLB_D2Q9) return RLB_E_ARG;
  if (o.correction != 0 && o.correction != 1) return RLB_E_ARG;
  if (o.ckpt_every != 0) return RLB_E_UNSUPPORTED;  // no tape: rlb_grad needs a handle
  if (o.correction && o.lattice != RLB_D2Q9) return RLB_E_UNSUPPORTED;
  if (p.nx < 1 || p.ny < 1 || p.nz < 1) return RLB_E_ARG;
  for (int k = 0; k < 3; ++k)
    if (p.bc[k] != RLB_PERIODIC && p.bc[k] != RLB_ZERO_GRADIENT) return RLB_E_ARG;
  if (o.lattice == RLB_D2Q9 && p.nz != 1) return RLB_E_ARG;
  if (!finite_tau(p.tau_f) || !finite_tau(p.tau_v) || !finite_tau(p.tau_e) ||
      !finite_tau(p.tau_eps) || std::isnan(p.tau_q) || (p.tau_q > 0.0 && !finite_tau(p.tau_q)))
    return RLB_E_TAU;
  if (!std::isfinite(p.eta_over_s) || p.eta_over_s < 0.0) return RLB_E_ARG;
  if (!(p.eos_gamma == 0.0 || (p.eos_gamma > 1.0 && p.eos_gamma <= 2.0))) return RLB_E_ARG;
  if (!std::isfinite(p.mass) || p.mass < 0.0) return RLB_E_ARG;
  if (p.eta_over_s > 0.0) {
    if (!std::isfinite(p.kappa) || !(p.kappa > 0.0)) return RLB_E_ARG;
    if (!std::isfinite(p.dof) || !(p.dof > 0.0)) return RLB_E_ARG;
    for (double a : {p.a_f, p.a_e, p.a_eps, p.a_q})
      if (!std::isfinite(a) || a < 0.0) return RLB_E_ARG;
  }
  if (o.correction && !paper_eos(p)) return RLB_E_UNSUPPORTED;
  return RLB_OK;
}

#define NA_HIP(call)                           \
  do {                                         \
    if ((call) != hipSuccess) return RLB_E_DEVICE; \
  } while (0)

// The run itself, with this device's scratch address in ws.
rlb_status run(unsigned char* ws, const rlb_params& p, const rlb_options& o, const double* n0,
               const double* eps0, const double* u0, int32_t nsteps, double* n, double* eps,
               double* P, double* gamma, double* u, double sums[5], int64_t* n_unphysical,
               hipStream_t st) {
  const bool d2 = o.lattice == RLB_D2Q9;
  const int64_t nc = (int64_t)p.nx * p.ny * p.nz;
  const Carve c = carve(nc, d2 ? 9 : 19, o.precision == RLB_FP32 ? 4 : 8);
  rlb::MemberDesc* d_desc = (rlb::MemberDesc*)(ws + c.desc);
  double* d_small = (double*)(ws + c.small);
  unsigned long long* d_count = (unsigned long long*)(d_small + 16);
  unsigned long long* d_bad_total = (unsigned long long*)(d_small + 20);
  unsigned long long* d_bad = (unsigned long long*)(ws + c.bad);
  double* d_parts = (double*)(ws + c.parts);
  double* d_xparts = (double*)(ws + c.xparts);
  void* buf[2] = {ws + c.buf0, ws + c.buf1};

  // the array keeps the previous call's contents: clear the counters
  const size_t nzero = (c.parts - c.small) / sizeof(unsigned long long);
  hipLaunchKernelGGL(k_zero, dim3(64), dim3(256), 0, st, (unsigned long long*)d_small, nzero);
  NA_HIP(hipGetLastError());

  rlb::MemberDesc desc;
  std::memset(&desc, 0, sizeof(desc));
  desc.offset = 0;
  desc.nx = p.nx;
  desc.ny = p.ny;
  desc.nz = p.nz;
  desc.ncells = (int32_t)nc;
  desc.bcx = p.bc[0];
  desc.bcy = p.bc[1];
  desc.bcz = p.bc[2];
  const double tq = p.tau_q > 0.0 ? p.tau_q : p.tau_v;
  desc.rt.w_f = 1.0 / p.tau_f;
  desc.rt.s_e = 1.0 / p.tau_e;
  desc.rt.s_eps = 1.0 / p.tau_eps;
  desc.rt.s_q = 1.0 / tq;
  desc.rt.s_v = 1.0 / p.tau_v;
  desc.ext.eta_s = p.eta_over_s;
  desc.ext.kappa = p.kappa;
  desc.ext.dof = p.dof;
  desc.ext.a_f = p.a_f;
  desc.ext.a_e = p.a_e;
  desc.ext.a_eps = p.a_eps;
  desc.ext.a_q = p.a_q;
  desc.ext.q_tied = p.tau_q > 0.0 ? 0 : 1;
  desc.ext.eos_gamma = p.eos_gamma > 0.0 ? p.eos_gamma : 4.0 / 3.0;
  desc.ext.mass = p.mass;
  desc.ext.general_eos = paper_eos(p) ? 0 : 1;
  const bool ext = p.eta_over_s > 0.0 || desc.ext.general_eos;
  NA_HIP(hipMemcpyAsync(d_desc, &desc, sizeof(desc), hipMemcpyHostToDevice, st));

  // validation of the input fields (rlb_init's checks), before any state
  NA_HIP(rlb::launch_validate(n0, eps0, u0, nc, d2 ? 1 : 0, d_desc, 1, d_count, st));
  unsigned long long cnt = 0;
  NA_HIP(hipMemcpyAsync(&cnt, d_count, sizeof(cnt), hipMemcpyDeviceToHost, st));
  NA_HIP(hipStreamSynchronize(st));
  if (cnt) return RLB_E_UNPHYSICAL;

  // t = 0: reference state and equilibria (rlb_init)
  NA_HIP(rlb::launch_member_refs(d_desc, 1, n0, eps0, u0, nc, d_parts, st));
  NA_HIP(d2 ? rlb::d2q9_launch_init(o.precision, buf[0], c.cs, d_desc, 1, n0, eps0, u0, nc, st)
            : rlb::launch_init(o.precision, buf[0], c.cs, d_desc, 1, n0, eps0, u0, nc, st));
  NA_HIP(hipMemcpyAsync(&desc, d_desc, sizeof(desc), hipMemcpyDeviceToHost, st));
  NA_HIP(hipStreamSynchronize(st));

  // steps (rlb_step): one fused launch per step, the default lattice variant
  rlb::LatticeGeom g{};
  g.nx = desc.nx;
  g.ny = desc.ny;
  g.nz = desc.nz;
  g.bcx = desc.bcx;
  g.bcy = desc.bcy;
  g.bcz = desc.bcz;
  g.cs = c.cs;
  g.rt = desc.rt;
  g.ref = desc.ref;
  g.ext = desc.ext;
  g.cached_store = 1;  // at most RLB_NOALLOC_SCRATCH_BYTES of state
  const int variant = d2 ? 2 : 3;
  int cur = 0;
  for (int32_t i = 0; i < nsteps; ++i) {
    if (d2)
      NA_HIP(rlb::d2q9_launch_step_lattice(o.precision, variant, false, o.correction != 0, ext,
                                           buf[cur], buf[1 - cur], g, d_parts, d_bad, st));
    else
      NA_HIP(rlb::launch_step_lattice(o.precision, variant, false, ext, buf[cur], buf[1 - cur],
                                      g, d_parts, d_bad, st));
    cur = 1 - cur;
  }

  // fields and lattice sums of the final state (rlb_moments)
  if (d2)
    NA_HIP(rlb::d2q9_launch_export(o.precision, buf[cur], c.cs, d_desc, 1, nc, n, eps, P, gamma,
                                   u, d_xparts, c.export_parts, st));
  else
    NA_HIP(rlb::launch_export(o.precision, buf[cur], c.cs, d_desc, 1, nc, n, eps, P, gamma, u,
                              d_xparts, c.export_parts, st));
  NA_HIP(rlb::launch_reduce(d_xparts, c.export_parts, d_small, st));
  NA_HIP(rlb::launch_sum_bad(d_bad, d_bad_total, st));
  double hs[5];
  unsigned long long bad = 0;
  NA_HIP(hipMemcpyAsync(hs, d_small, sizeof(hs), hipMemcpyDeviceToHost, st));
  NA_HIP(hipMemcpyAsync(&bad, d_bad_total, sizeof(bad), hipMemcpyDeviceToHost, st));
  NA_HIP(hipStreamSynchronize(st));
  if (sums) std::memcpy(sums, hs, sizeof(hs));
  if (n_unphysical) *n_unphysical = (int64_t)bad;
  return bad ? RLB_E_UNPHYSICAL : RLB_OK;
}

}  // namespace

extern "C" rlb_status rlb_run_noalloc(const rlb_params* member, const rlb_options* opt,
                                      const double* n0, const double* eps0, const double* u0,
                                      int32_t nsteps, double* n, double* eps, double* P,
                                      double* gamma, double* u, double sums[5],
                                      int64_t* n_unphysical, void* hip_stream) {
  if (!member || !opt || !n0 || !eps0 || !u0 || nsteps < 0) return RLB_E_ARG;
  rlb_status s = check(*member, *opt);
  if (s != RLB_OK) return s;
  const int64_t nc = (int64_t)member->nx * member->ny * member->nz;
  if (nc >= (int64_t(1) << 31)) return RLB_E_SCRATCH;
  const Carve c = carve(nc, opt->lattice == RLB_D2Q9 ? 9 : 19,
                        opt->precision == RLB_FP32 ? 4 : 8);
  if (c.total > (size_t)RLB_NOALLOC_SCRATCH_BYTES) return RLB_E_SCRATCH;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RLB_E_DEVICE;
  DeviceSlot& slot = g_slots[dev];
  std::lock_guard<std::mutex> lock(slot.mu);
  if (!slot.ptr) {  // first call on this device (it is current): this copy's address
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
      return RLB_E_DEVICE;
    slot.ptr = (unsigned char*)ptr;
  }
  return run(slot.ptr, *member, *opt, n0, eps0, u0, nsteps, n, eps, P, gamma, u, sums,
             n_unphysical, (hipStream_t)hip_stream);
}
