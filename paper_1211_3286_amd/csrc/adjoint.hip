// Tape and adjoint of the g update (rlb_grad).

#include <hip/hip_runtime.h>

#include "adjoint.hpp"

namespace rlb {

namespace {
size_t al(size_t v) { return (v + 255) / 256 * 256; }
}  // namespace

TapeLayout tape_layout(int64_t ncells, int64_t cs, size_t esz, int K, int tape_steps,
                       int max_parts) {
  TapeLayout L;
  L.K = K;
  L.gbytes = 19 * (size_t)cs * esz;
  L.n_ckpt = tape_steps / K + 1;
  L.max_parts = max_parts;
  size_t o = 0;
  L.off_ckpt = o;
  o = al(o + L.gbytes * L.n_ckpt);
  L.off_seg = o;
  o = al(o + L.gbytes * K);
  L.off_adj = o;
  o = al(o + 2 * L.gbytes);
  L.off_fields = o;
  o = al(o + sizeof(double) * 4 * (size_t)ncells);
  L.off_tparts = o;
  o = al(o + sizeof(double) * 5 * (size_t)max_parts);
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
  (void)t;
  (void)c;
  (void)dL_du;
  (void)dL_deps;
  (void)dL_dtau;
  (void)dL_deps0;
  (void)dL_du0;
  (void)io_on_device;
  return RLB_E_UNSUPPORTED;
}

void tape_release(Tape& t) { t.base = nullptr; }

}  // namespace rlb
