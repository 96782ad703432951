/*
 * rlb.h - C ABI of the MI355X (gfx950) relativistic lattice Boltzmann step.
 *
 * Model: Q. Li, K. H. Luo, X. J. Li, "Lattice Boltzmann method for relativistic
 * hydrodynamics: issues on conservation law of particle number and
 * discontinuities" (arXiv:1211.3286), Sec. II and Sec. V.A. Two distributions
 * per cell on the D3Q19 lattice:
 *   f  particle number,   BGK collision with tau_f      (Eq. 5, f_eq Eq. 7)
 *   g  energy-momentum,   MRT collision, Lambda = M^-1 S M (Eqs. 30, 31, 35;
 *                         g_eq Eqs. 8-9), relaxation times tau_v (shear rows),
 *                         tau_e (energy/bulk row), tau_eps (energy-square row),
 *                         tau_q (ghost rows); tau_sigma = tau_j = dt.
 * Macroscopic fields (Eq. 10): n gamma = sum f, (eps + P) gamma^2 - P = sum g,
 * (eps + P) gamma^2 u = sum e g, with the equation of state P = eps / 3.
 * The recovery of (n, eps, P, gamma, u) from these sums, the conservation sums
 * and every reduction are done in FP64 whatever the population precision.
 *
 * Lattice units: dt = dx = c = 1, c_s^2 = 1/3.
 *
 * Velocity order (index a of every population array):
 *   0: (0,0,0)
 *   1: (+1,0,0)  2: (-1,0,0)  3: (0,+1,0)  4: (0,-1,0)  5: (0,0,+1)  6: (0,0,-1)
 *   7: (+1,+1,0) 8: (-1,-1,0) 9: (+1,-1,0) 10: (-1,+1,0)
 *  11: (+1,0,+1) 12: (-1,0,-1) 13: (+1,0,-1) 14: (-1,0,+1)
 *  15: (0,+1,+1) 16: (0,-1,-1) 17: (0,+1,-1) 18: (0,-1,+1)
 *
 * The D2Q9 model (rlb_options.lattice = RLB_D2Q9) is the MRT model the paper
 * runs in Sec. V (Eqs. 30-35): S = diag(1/tau_sigma, 1/tau_e, 1/tau_eps,
 * 1/tau_j, 1/tau_q, 1/tau_j, 1/tau_q, 1/tau_v, 1/tau_v) (Eq. 31), g_eq of
 * Eqs. (32)-(33), moment equilibria Eq. (34); f keeps the BGK of Eq. (5) with
 * f_eq of Eq. (7)'s form and the D2Q9 weights 4/9, 1/9, 1/36. Its lattices
 * are nx x ny x 1 (velocities in the x-y plane, u_z = 0); velocity order:
 *   0: (0,0)  1: (+1,0)  2: (0,+1)  3: (-1,0)  4: (0,-1)
 *   5: (+1,+1)  6: (-1,+1)  7: (-1,-1)  8: (+1,-1)
 * and every "19" below reads 9 for it.
 *
 * Field layout: a lattice of nx*ny*nz cells, x fastest: cell = x + nx*(y + ny*z).
 * A batch of members ("n_members" lattices, e.g. shock tubes of uneven
 * length) is packed member after member; member m starts at the prefix sum of
 * the cell counts of members 0..m-1. Scalar fields are arrays of that many
 * doubles; a velocity field is three such planes (u_x, u_y, u_z).
 *
 * Time: the state after step t holds the post-collision populations at t;
 * rlb_init sets the state at t = 0 to the equilibria of the given fields.
 * One rlb_step advances every cell by: streaming (pull from x - e_a, with
 * periodic wrap or zero-gradient clamp per axis), the Eq. (10) sums, the
 * recovery, the equilibria, the f BGK and g MRT collisions.
 *
 * Ownership: the caller owns every buffer. The library never allocates device
 * memory: all device state lives in the caller's workspace, whose size
 * rlb_workspace_size reports, and which must stay valid (and untouched by the
 * caller) until rlb_free. All device work is enqueued on the caller's HIP
 * stream given to rlb_init (NULL = the null stream); calls that return host
 * data synchronise that stream. Pointers marked "device" must be device
 * memory of the device that was current at rlb_init; "host" pointers are
 * ordinary host memory. A handle must not be used from two threads at once.
 *
 * Errors: every call returns an rlb_status; nothing is thrown and nothing
 * exits. A failed call leaves the state as it was unless stated otherwise.
 */
#ifndef RLB_H
#define RLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RLB_OK = 0,
  RLB_E_ARG = -1,         /* NULL pointer, bad size, bad enum, bad dims */
  RLB_E_TAU = -2,         /* a relaxation time <= 1/2 (negative viscosity) or not finite */
  RLB_E_UNPHYSICAL = -3,  /* an input cell has eps <= 0, n < 0 or |u| >= 1; or cells
                             became inadmissible (E <= 0 or |M| >= E) during steps */
  RLB_E_WORKSPACE = -4,   /* workspace NULL, misaligned (needs 256 B) or too small */
  RLB_E_DEVICE = -5,      /* a HIP runtime call failed */
  RLB_E_STATE = -6,       /* call not valid in this state (e.g. rlb_grad without tape) */
  RLB_E_UNSUPPORTED = -7, /* valid request the library does not provide (e.g.
                             tube rounds for a batch that is not all 1 x 1 x L) */
  RLB_E_SCRATCH = -8      /* rlb_run_noalloc: the lattice does not fit the fixed
                             scratch array of RLB_NOALLOC_SCRATCH_BYTES */
} rlb_status;

enum { RLB_PERIODIC = 0, RLB_ZERO_GRADIENT = 1 };
enum { RLB_FP64 = 0, RLB_FP32 = 1 };
enum { RLB_D3Q19 = 0, RLB_D2Q9 = 1 };

/* One lattice (or one member of a batch). */
typedef struct {
  int32_t nx, ny, nz;  /* cells per axis, each >= 1 */
  int32_t bc[3];       /* RLB_PERIODIC or RLB_ZERO_GRADIENT for x, y, z. Zero-gradient
                          is the reading of the paper's "open" boundaries: the pull
                          source coordinate is clamped into [0, N-1]. */
  double tau_f;        /* f relaxation time, Eq. (5) */
  double tau_v;        /* shear rows (3p_xx, p_ww, p_xy, p_yz, p_xz), Eq. (31) */
  double tau_e;        /* energy row e (bulk viscosity), Eq. (31) */
  double tau_eps;      /* energy-square row eps, Eq. (31) */
  double tau_q;        /* ghost rows (q, 3pi_xx, pi_ww, m; D2Q9: the q rows of
                          Eq. 31); <= 0 means tau_q = tau_v */
  /* Relaxation times from the ratio eta/s, cell by cell and step by step
   * (Sec. III.B), when eta_over_s > 0 (0 = off, the fixed taus above apply):
   *   T = P / n (ideal gas), n_eq = dof T^3 / pi^2, s = 4n - n ln(n / n_eq),
   *   tau_v = 1/2 + kappa (eta/s) s / (c_s^2 (eps + P) gamma)
   * (the viscosity relation after Eq. 10 solved for tau, kappa the shear-
   * viscosity transformation of Secs. IV and V.A, 1 = none), and for x in
   * {f, e, eps, q} with a_x > 0: tau_x - 1/2 = a_x (tau_v - 1/2); tau_q <= 0
   * ties tau_q to the local tau_v. A cell with n <= 0 or P <= 0 uses the
   * fixed taus, which must be valid in any case. Not with a tape or the
   * segmented launches (RLB_E_UNSUPPORTED). T = P / n is the ideal-gas
   * temperature, also under the general equation of state below. */
  double eta_over_s;   /* >= 0 */
  double kappa;        /* > 0 when eta_over_s > 0 */
  double dof;          /* degeneracy d_G > 0 (16 for gluons) */
  double a_f, a_e, a_eps, a_q;  /* >= 0 */
  /* Equation of state P = (eos_gamma - 1)(eps - mass n) (an extension of the
   * paper's P = eps/3, which is eos_gamma 0 or 4/3 with mass 0). Eq. (10) then
   * leaves one equation for z = (eps + P) gamma^2, solved per cell by a
   * bracketed Newton iteration in FP64. eos_gamma in (1, 2] (or 0), mass >= 0;
   * every input cell needs eps > mass n; cells whose root gives P <= 0 are
   * inadmissible. Not with a tape, the correction term or the segmented
   * launches (RLB_E_UNSUPPORTED). */
  double eos_gamma;
  double mass;
} rlb_params;

typedef struct {
  int32_t precision;   /* RLB_FP32 or RLB_FP64: storage and collision precision of
                          the populations. Recovery, moment sums and reductions are
                          FP64 in both. */
  int32_t ckpt_every;  /* 0: no tape. K > 0: keep the g populations every K steps
                          so that rlb_grad can run (single-member handles only). */
  int32_t tape_steps;  /* with ckpt_every > 0: the largest step count rlb_grad can
                          differentiate (steps taken beyond it disable rlb_grad). */
  int32_t diag_every;  /* 0: none. D > 0: every D-th step (and the last step of each
                          rlb_step call) also leaves per-block FP64 partial sums of
                          the conservation moments, read by rlb_diagnostics. */
  int32_t lattice;     /* RLB_D3Q19 (0) or RLB_D2Q9 (1). D2Q9: every member has
                          nz = 1 and every input cell u_z = 0 (else RLB_E_ARG,
                          RLB_E_UNPHYSICAL); no tape (ckpt_every > 0 gives
                          RLB_E_UNSUPPORTED). */
  int32_t correction;  /* 0 or 1 (D2Q9 only, else RLB_E_UNSUPPORTED): add the
                          correction term of Eqs. (37)-(38) to the p_xx row,
                          m* = m - S (m - m_eq) + (I - S/2) C, C_7 from central
                          y-differences of the recovered fields of each cell's
                          y-neighbours (flows along y, the paper's z). The
                          printed C_7 belongs to the row e_flow^2 - e_perp^2,
                          the negative of this basis' e_x^2 - e_y^2, so the
                          row receives -C_7. No correction next to an
                          inadmissible cell. */
} rlb_options;

typedef struct rlb_sim* rlb_handle;

/* Bytes of device workspace rlb_init needs for these members and options.
 * members: host array of n_members (>= 1) lattices. opt: host, non-NULL. */
rlb_status rlb_workspace_size(const rlb_params* members, int32_t n_members,
                              const rlb_options* opt, size_t* bytes);

/* Create a simulation and set the state at t = 0 to the equilibria of the
 * initial fields: f = f_eq(n0, u0) (Eq. 7), g = g_eq(eps0, P0, u0)
 * (Eqs. 8-9), P0 = eps0/3 (or the general equation of state of rlb_params).
 *   n0, eps0: ncells doubles each; u0: 3 * ncells doubles (u_x, u_y, u_z planes).
 *   fields_on_device: 1 if n0/eps0/u0 are device pointers, 0 for host.
 *   workspace: device, 256-byte aligned, at least rlb_workspace_size bytes.
 *   hip_stream: hipStream_t (NULL = null stream); every later call uses it.
 * Validation (before any state is written): dims >= 1, bc in {0, 1}, every
 * tau > 1/2 and finite, the eta/s and equation-of-state parameters in range
 * (RLB_E_ARG, RLB_E_TAU); every cell n0 >= 0, eps0 > 0, |u0| < 1 (finite),
 * eps0 > mass n0 under the general equation of state, u_z = 0 on D2Q9
 * (RLB_E_UNPHYSICAL); a member of 2^31 cells or more, or an option
 * combination listed as unsupported above (RLB_E_UNSUPPORTED). On error *out
 * is NULL. The fields are only read during this call. */
rlb_status rlb_init(rlb_handle* out, const rlb_params* members, int32_t n_members,
                    const rlb_options* opt, const double* n0, const double* eps0,
                    const double* u0, int32_t fields_on_device, void* workspace,
                    size_t workspace_bytes, void* hip_stream);

/* Advance every member by nsteps >= 0 steps, asynchronously on the stream.
 * One step of a cell is the update of Sec. II and V.A: streaming, the left-
 * hand side of Eqs. (5), (6) and (35) (pull from x - e_a); the moments of
 * Eq. (10) and the recovery of (n, eps, P, gamma, u) from them; the
 * equilibria of Eqs. (7)-(9) (D2Q9: Eqs. 32-34); the f BGK collision of
 * Eq. (5) and the g MRT collision of Eqs. (30)-(31), m* = m - S(m - m_eq),
 * g* = M^-1 m* (Eq. 35), with the correction of Eq. (37) when selected.
 * Single-member lattices run one fused kernel launch per step (D2Q9: or
 * rounds of H steps on tiles held in LDS); batches (and small single
 * lattices) run in a HIP graph, either all nsteps inside one persistent
 * launch, or as rounds of H steps on segments held in LDS (1 x 1 x L tubes;
 * narrow D2Q9 members cut into rows), by the selected variant (rlb_tune picks
 * the fastest). The variants give identical results, bit for bit. No
 * validation per step: cells that
 * become inadmissible (E <= 0 or |M| >= E) keep their populations uncollided
 * and are counted; the count is reported by rlb_moments/rlb_diagnostics. */
rlb_status rlb_step(rlb_handle h, int32_t nsteps);

/* Fields of the current state (Eq. 10 sums + recovery, FP64) and the lattice
 * sums {sum n gamma, sum (sigma - P), sum sigma u_x, sum sigma u_y, sum sigma u_z}.
 * Any output pointer may be NULL (skipped). Scalar outputs: ncells doubles;
 * u: 3 * ncells. out_on_device: 1 if the field pointers are device memory
 * (sums and n_unphysical are always host). n_unphysical: host int64, the
 * number of inadmissible cell-updates since rlb_init (their fields are NaN).
 * Synchronises the stream. Returns RLB_E_UNPHYSICAL when that count is > 0
 * (outputs are still written). */
rlb_status rlb_moments(rlb_handle h, double* n, double* eps, double* P, double* gamma,
                       double* u, double sums[5], int64_t* n_unphysical,
                       int32_t out_on_device);

/* FP64 lattice sums of the latest diagnostics step (see diag_every), and the
 * step index they belong to (the sums of the populations streamed into that
 * step, i.e. the conserved totals after it up to rounding). Host outputs;
 * synchronises. RLB_E_STATE if no diagnostics step has run. */
rlb_status rlb_diagnostics(rlb_handle h, double sums[5], int64_t* step,
                           int64_t* n_unphysical);

/* Copy the current populations out as FP64: f and g are each 19 * ncells
 * doubles, population a of cell c at [a * ncells + c]. Either may be NULL.
 * out_on_device as in rlb_moments. Synchronises. */
rlb_status rlb_populations(rlb_handle h, double* f, double* g, int32_t out_on_device);

/* Adjoint of the whole run (rlb_init + every rlb_step since), by reverse
 * sweeps over checkpointed segments with recomputation. Given the gradient
 * of a loss with respect to the current velocity and energy density fields,
 *   dL_du: 3 * ncells, dL_deps: ncells,
 * returns dL_dtau = {dL/dtau_v, dL/dtau_e, dL/dtau_eps} (host, 3 doubles),
 * dL_deps0 (ncells) and dL_du0 (3 * ncells) for the initial fields.
 * tau_q <= 0 ties the ghost rows to tau_v, and then their contribution is part
 * of dL/dtau_v. Only g enters (u and eps never depend on f). io_on_device as
 * in rlb_moments. Requires ckpt_every > 0 and steps taken <= tape_steps,
 * else RLB_E_STATE. Does not change the forward state. Synchronises. */
rlb_status rlb_grad(rlb_handle h, const double* dL_du, const double* dL_deps,
                    double dL_dtau[3], double* dL_deps0, double* dL_du0,
                    int32_t io_on_device);

/* Kernel variants (block shape x cells per thread; for the lattice step also
 * the waves per SIMD: a name ending in "/w3" reserves unused LDS so that 3
 * waves per SIMD run instead of 4; for round kernels the steps per launch,
 * "/hH") of the path this handle dispatches to. rlb_tune times every variant with HIP events on trial steps
 * that read the current state and write only the spare buffer (the state is
 * unchanged), selects the fastest, and returns all timings (ms per step,
 * host array of rlb_num_variants doubles, may be NULL). */
rlb_status rlb_num_variants(rlb_handle h, int32_t* count);
rlb_status rlb_variant_name(rlb_handle h, int32_t variant, char* buf, size_t buflen);
rlb_status rlb_set_variant(rlb_handle h, int32_t variant);
rlb_status rlb_get_variant(rlb_handle h, int32_t* variant);
rlb_status rlb_tune(rlb_handle h, int32_t trial_steps, int32_t* best_variant,
                    double* ms_per_step);

/* Step count since rlb_init, and the name of the kernel rlb_step launches. */
rlb_status rlb_info(rlb_handle h, int64_t* steps, char* kernel_name, size_t buflen);

/* Release the handle (no device memory is freed: the workspace is the
 * caller's). Waits for the handle's queued work. NULL is ignored. */
void rlb_free(rlb_handle h);

const char* rlb_status_string(rlb_status s);

/* ---------------------------------------------------------------------------
 * Allocation-free run, for callers that cannot allocate memory: tight serving
 * or sweep loops, harnesses that forbid allocation, callers that hold no
 * workspace. It does what rlb_init + rlb_step(nsteps) + rlb_moments do on
 * one lattice (single member, fixed options), with the same kernels, and
 * allocates nothing: no device or host memory, no handle, no HIP graph.
 *
 * Everything besides the caller's fields (the two population buffers, the
 * member descriptor, the partial sums and the inadmissible-cell counters)
 * lives in one fixed device array of RLB_NOALLOC_SCRATCH_BYTES inside the
 * library. Each device the call runs on holds its own copy of that array
 * until the process ends. A lattice whose state does not fit it returns
 * RLB_E_SCRATCH before any device work: about 2 x 2 x 19 x sizeof(precision)
 * bytes per cell on D3Q19 (2 x 2 x 9 x ... on D2Q9), e.g. up to about 220,000
 * cells in FP32 and 110,000 in FP64 on D3Q19.
 *
 * The array is shared by every call on a device and keeps the last call's
 * contents; each call clears its counters first. Calls on one device are
 * serialised by a lock inside the library (each call waits for its own stream
 * before it returns), so threads of one process may call it concurrently;
 * device work of another process has its own copy.
 *
 *   member, opt: host. opt->ckpt_every must be 0 (else RLB_E_UNSUPPORTED);
 *     opt->diag_every and opt->tape_steps are ignored; every other option and
 *     parameter as for rlb_init (same checks, same status codes).
 *   n0, eps0, u0: device, the initial fields (layout of rlb_init), read only.
 *   nsteps >= 0: steps to advance.
 *   n, eps, P, gamma, u: device outputs of the fields after nsteps, as
 *     rlb_moments with out_on_device = 1; any may be NULL.
 *   sums: host, 5 doubles or NULL; n_unphysical: host or NULL (as rlb_moments).
 *   hip_stream: hipStream_t (NULL = null stream); the call synchronises it.
 * Returns RLB_E_UNPHYSICAL for inadmissible input cells (nothing computed) or
 * cells that became inadmissible (outputs written, as rlb_moments). */
#define RLB_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
rlb_status rlb_run_noalloc(const rlb_params* member, const rlb_options* opt,
                           const double* n0, const double* eps0, const double* u0,
                           int32_t nsteps, double* n, double* eps, double* P, double* gamma,
                           double* u, double sums[5], int64_t* n_unphysical,
                           void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* RLB_H */
