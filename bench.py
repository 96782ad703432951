#!/usr/bin/env python3
"""Throughput of the relativistic MRT lattice Boltzmann step on one MI355X.

Headline workload: a 256^3 periodic lattice (D3Q19, two distributions), smooth
random flow from 16 Fourier modes (|k| <= 4, max|u| = 0.1, eps and n = 1 +
0.05 noise, seed 1211), tau_v = 0.8, tau_e = 0.55, tau_eps = 0.7, tau_f = 0.8,
FP32 populations with FP64 recovery and FP64 conservation sums fused into
every step. One timed step = one fused kernel launch over all 16.8M cells.

Also reported ("forms"): the same step in FP64, the 1 x 1 x 800 FP64 shock
tube (2000 steps), the batch of 64 ragged shock tubes (3000 steps, one HIP
graph launch whose kernel nodes are rounds of H steps: kernel_nodes states
how many), the adjoint gradient of a 512 x 512 run (1000 steps, checkpoints
every 50), the 512^3 blast, the D2Q9 MRT model of Sec. V (a 4096^2 lattice,
the 4 x 800 Cases A-D batch, the correction of Eqs. 37-38), and relaxation
times set per cell from eta/s. Every form states its error: a short live run
of the timed kernel variant against the FP64 oracle from the same input
(error_vs_oracle), and for the adjoint the error of dL/dtau against central
finite differences and of every output against the oracle's own adjoint.

Prints one JSON line. ``value`` is MLUPS (million lattice-cell updates per
second) with the populations resident in HBM; ``roofline`` prices the fused
kernel at its algorithmic traffic (2 x 38 populations per cell update);
``cpu_baseline`` times the FP64 CPU oracle on a bounded sample of the same
workload on the host cores; ``error_vs_oracle`` then runs the GPU path from
the same input for the same number of steps, in the kernel variants that were
timed, and gives its max-norm errors against that oracle state over all
cells.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS + % HBM roofline, FP32 vs FP64 step, batched and adjoint, at stated error"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
D2Q9_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_d2q9.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_d2q9.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1211_3286_amd", "csrc", f)
                  for f in ("cell.hpp", "device_util.hpp", "internal.hpp", "kernels.hip",
                            "api.cpp")]
D2Q9_SOURCES = [os.path.join(ROOT, "paper_1211_3286_amd", "csrc", f)
                for f in ("cell.hpp", "cell2d.hpp", "device_util.hpp", "internal.hpp",
                          "kernels2d.hip", "api.cpp")]
# MI355X: 256 CUs at 2.4 GHz, each issuing at most one wave64 VALU
# instruction a cycle (4 SIMDs, 4 cycles per wave64 instruction)
VALU_PEAK_GINST = 256 * 2.4


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash(sources=None) -> str:
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _record(path: str, kernel: str):
    """A kernel's entry of a committed D2Q9 counter record, if the record
    still describes the current D2Q9 sources (else None)."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        db = json.load(fh)
    if db.get("source_hash") != kernel_hash(D2Q9_SOURCES):
        return None
    return db.get("kernels", {}).get(kernel)


def measured_d2q9(kernel: str):
    return _record(D2Q9_TRAFFIC_FILE, kernel)


def measured_valu(kernel: str):
    return _record(VALU_FILE, kernel)


def measured_traffic(kernel: str, cells: int):
    """HBM bytes per launch from the committed PMC summary, if it still
    describes the current kernel source (else None). The occupancy-capped
    forms (".../w3") launch the same instantiation and move the same bytes;
    the counters, which see instantiations, hold one record for both."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        db = json.load(fh)
    rec = db.get(kernel.split("/")[0])
    if not rec or rec.get("source_hash") != kernel_hash() or rec.get("cells") != cells:
        return None
    return rec.get("bytes_per_launch")


def time_steps(torch, sim, steps: int, warmup: int):
    if warmup:
        sim.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def copy_calibration(torch, nbytes: int = 1 << 30, reps: int = 5):
    """A plain device-to-device copy of known size: its byte counters give the
    scale of the FETCH_SIZE / WRITE_SIZE counters of the step kernel."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"bytes_read": nbytes, "bytes_written": nbytes, "ms": ms,
            "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}


def bench_lattice(torch, rlb, wl, n: int, precision: int, steps: int, warmup: int,
                  diag_every: int):
    prob = wl.random_modes(n, seed=1211, umax=0.1, amp=0.05, tau_v=0.8, tau_e=0.55,
                           tau_eps=0.7, tau_f=0.8)
    sim = rlb.from_problems(prob, precision=precision, diag_every=diag_every)
    # the two best block shapes differ by about 0.5 %: 30 timed trial steps
    # per variant keep the choice above the run-to-run noise
    tune = sim.tune(trial_steps=30)
    log("tuned", tune["name"], {k: round(v, 4) for k, v in tune["ms_per_step"].items()})
    s0 = sim.sums()
    ms, wall = time_steps(torch, sim, steps, warmup)
    s1 = sim.sums()
    diag, dstep, bad = sim.diagnostics()
    cells = prob.params.ncells
    bytes_per_cell = 2 * 38 * (4 if precision == rlb.FP32 else 8)
    drift = float(abs(s1 - s0).max() / abs(s0[:2]).max())
    out = {"ms_per_step": ms, "mlups": cells / (ms * 1e-3) / 1e6, "cells": cells,
           "kernel": sim.kernel_name, "bytes_per_cell": bytes_per_cell,
           "achieved_gbs": bytes_per_cell * cells / (ms * 1e-3) / 1e9,
           "conservation_drift": drift, "inadmissible": bad, "wall_s": wall,
           "variant_ms": tune["ms_per_step"], "problem": prob}
    out["frac"] = out["achieved_gbs"] / HBM_PEAK_GBS
    sim.close()
    return out


def graph_shape(kernel: str, steps: int) -> dict:
    """What one rlb_step of a persistent-path variant launches: the tube and
    strip rounds are a HIP graph of ceil(steps / H) kernel nodes (H steps
    each, from the variant name's /hH); the one-block and segmented kernels
    are one node doing every step."""
    m = re.search(r"/h(\d+)", kernel)
    h = int(m.group(1)) if m else None
    return {"graph_launches": 1, "kernel_nodes": -(-steps // h) if h else 1,
            "steps_per_node": h if h else steps}


def live_error(torch, rlb, problems, steps: int, precision: int, kernel, **kw):
    """Max-norm errors of a short GPU run (the kernel variant that was timed)
    against the FP64 oracle from the same input: populations, n, eps over
    every cell (max|a - b| / max|b| per array) and u (max|a - b|), each the
    worst over the members; plus the inadmissible count of each side."""
    import numpy as np
    import oracle
    if not isinstance(problems, (list, tuple)):
        problems = [problems]
    sim = rlb.from_problems(problems, precision=precision, **kw)
    sim.variant = kernel if isinstance(kernel, int) else sim.variants().index(kernel)
    sim.step(steps)
    f, g = sim.populations()
    m = sim.moments(allow_unphysical=True)
    f, g = f.cpu().numpy(), g.cpu().numpy()
    gpu = {k: m[k].cpu().numpy() for k in ("n", "eps", "u")}
    sim.close()
    err = {"steps": steps, "cells": int(sum(p.params.ncells for p in problems))}
    worst = dict.fromkeys(("f", "g", "n", "eps", "u"), 0.0)
    bad_o = 0
    off = 0
    for p in problems:
        st = oracle.run(p, steps)
        F = st.fields()
        bad_o += st.bad
        nc = p.params.ncells
        sl = slice(off, off + nc)
        pairs = {"f": (f[:, sl], st.f.reshape(f.shape[0], nc)),
                 "g": (g[:, sl], st.g.reshape(g.shape[0], nc)),
                 "n": (gpu["n"][sl], F["n"].ravel()), "eps": (gpu["eps"][sl], F["eps"].ravel()),
                 "u": (gpu["u"][:, sl], F["u"].reshape(3, nc))}
        for k, (a, b) in pairs.items():
            keep = np.isfinite(a) & np.isfinite(b)
            if not keep.any():
                continue
            d = np.abs(a[keep] - b[keep]).max()
            worst[k] = max(worst[k], float(d if k == "u" else d / np.abs(b[keep]).max()))
        off += nc
    err.update(worst)
    err["inadmissible_gpu"], err["inadmissible_oracle"] = m["bad"], int(bad_o)
    return err


def bench_batched(torch, rlb, wl, steps: int = 3000, check_steps: int = 200):
    tubes = wl.tube_batch()
    sim = rlb.from_problems(tubes, precision=rlb.FP32)
    tune = sim.tune(trial_steps=50)
    log("batched tuned", tune["name"], {k: round(v, 5) for k, v in tune["ms_per_step"].items()})
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cells = sum(t.params.ncells for t in tubes)
    m = sim.moments(allow_unphysical=True)
    res = {"tubes": len(tubes), "steps": steps, "cells": cells, "ms_total": ms,
           "tube_steps_per_s": len(tubes) * steps / (ms * 1e-3),
           "mlups": cells * steps / (ms * 1e-3) / 1e6,
           "effective_gbs": 304 * cells * steps / (ms * 1e-3) / 1e9,
           "kernel": sim.kernel_name, **graph_shape(sim.kernel_name, steps),
           "inadmissible": m["bad"],
           "note": "working set ~35 MB stays in L2/MALL; effective GB/s is not HBM traffic"}
    sim.close()
    # every tube against the oracle over a short run of the timed variant (the
    # tests hold the 3000-step per-tube errors)
    res["error_vs_oracle"] = live_error(torch, rlb, tubes, check_steps, rlb.FP32, res["kernel"])
    return res


def bench_shock_tube(torch, rlb, wl, steps: int = 2000, dump_every: int = 200):
    """The 1 x 1 x 800 FP64 shock tube (zero-gradient long axis, tau = 0.9):
    GPU steps per second over 2000 steps in one rlb_step call (the tuned
    persistent variant), and the max-norm error against the oracle at every
    dump of a second run stopped every 200 steps; the same in FP32."""
    import numpy as np
    import oracle
    prob = wl.shock_tube(800)
    st = oracle.State.init(prob)
    ref = []
    for _ in range(steps // dump_every):
        st.step(dump_every)
        F = st.fields()
        ref.append({"f": st.f.reshape(19, -1).copy(), "g": st.g.reshape(19, -1).copy(),
                    "n": F["n"].ravel(), "eps": F["eps"].ravel(), "u": F["u"].reshape(3, -1)})
    out = {"lattice": "1x1x800", "steps": steps, "dump_every": dump_every}
    for prec, name in ((rlb.FP64, "fp64"), (rlb.FP32, "fp32")):
        sim = rlb.from_problems(prob, precision=prec)
        tune = sim.tune(trial_steps=50)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        sim.close()
        # the dumps: a fresh run stopping every dump_every steps
        sim = rlb.from_problems(prob, precision=prec)
        sim.variant = sim.variants().index(tune["name"])
        worst = dict.fromkeys(("f", "g", "n", "eps", "u"), 0.0)
        for r in ref:
            sim.step(dump_every)
            f, g = sim.populations()
            m = sim.moments()
            gpu = {"f": f.cpu().numpy(), "g": g.cpu().numpy(), "n": m["n"].cpu().numpy(),
                   "eps": m["eps"].cpu().numpy(), "u": m["u"].cpu().numpy()}
            for k, a in gpu.items():
                d = np.abs(a - r[k]).max()
                worst[k] = max(worst[k], float(d if k == "u" else d / np.abs(r[k]).max()))
        sim.close()
        out[name] = {"ms_total": ms, "steps_per_s": steps / (ms * 1e-3),
                     "mlups": 800 * steps / (ms * 1e-3) / 1e6, "kernel": tune["name"],
                     **graph_shape(tune["name"], steps),
                     "error_vs_oracle_over_dumps": worst}
    return out


def bench_blast(torch, rlb, wl, L: int = 512, steps: int = 400, warmup: int = 10):
    """Moderately relativistic 3D blast, FP32, clamped faces (about 41 GB of
    double-buffered populations). As specified (100:1 pressure, max|u| = 0.6)
    the flow leaves the admissible range of the D3Q19 model within a few
    steps along the lattice diagonals; those cells are left uncollided and
    counted, and the count is reported with the throughput."""
    prob = wl.blast(L)
    sim = rlb.from_problems(prob, precision=rlb.FP32, diag_every=50)
    tune = sim.tune(trial_steps=5)
    del prob
    ms, wall = time_steps(torch, sim, steps, warmup)
    m = sim.moments(allow_unphysical=True)
    cells = L ** 3
    res = {"lattice": f"{L}x{L}x{L}", "steps": steps, "ms_per_step": ms,
           "mlups": cells / (ms * 1e-3) / 1e6, "kernel": tune["name"],
           "achieved_gbs": 304 * cells / (ms * 1e-3) / 1e9,
           "frac": 304 * cells / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "inadmissible_cell_updates": m["bad"],
           "inadmissible_fraction": m["bad"] / float(cells * (steps + warmup)),
           "max_u_admissible": float(torch.nan_to_num(m["u"].norm(dim=0), nan=0.0).max().item()),
           "workspace_gb": sim.ws_bytes / 1e9}
    variant = sim.variant
    sim.close()
    del m
    torch.cuda.empty_cache()
    # the FP64 oracle of 512^3 needs more host memory than the box holds: the
    # error is stated on the 128^3 analogue (sphere radius 16), 20 steps, in
    # the timed block shape, FP64 (the parity check: admissibility decided on
    # the same inputs) and FP32 (populations can leave the admissible range
    # at other cells than in FP64; the counts say how many)
    small = wl.blast(128)
    res["error_vs_oracle_128"] = {
        "fp64": live_error(torch, rlb, small, 20, rlb.FP64, variant),
        "fp32": live_error(torch, rlb, small, 20, rlb.FP32, variant)}
    return res


def bench_adjoint(torch, rlb, wl, L: int = 512, steps: int = 1000, K: int = 50,
                  oracle_L: int = 64, oracle_steps: int = 200, grad_reps: int = 5):
    """The adjoint form on the L x L x 1 shear-wave/vortex field, FP32, with
    checkpoints every K steps. The loss is the L2 mismatch of the final u and
    eps with a target made by the same model (FP64) at seeded perturbed
    relaxation times plus 1 % noise. Times (HIP events on the handle's
    stream): the taped forward in the autotuned step variant, and the
    gradient (rlb_grad): the median of
    grad_reps calls after one untimed call that instantiates its graph.
    Errors: dL/dtau against central finite differences of the FP64 forward
    (h = 1e-4), over max(|FD|, |grad|); and
    every output against the oracle's FP64 adjoint on the oracle_L^2 instance,
    oracle_steps steps."""
    import copy
    import numpy as np
    import oracle
    prob = wl.shear_vortex(L)
    p = prob.params
    nc = p.ncells

    def fields_fp64(q):
        sim = rlb.from_problems(q, precision=rlb.FP64)
        sim.step(steps)
        m = sim.moments()
        out = (m["u"].cpu().numpy(), m["eps"].cpu().numpy())
        sim.close()
        return out

    def with_tau(**kw):
        q = copy.deepcopy(prob)
        for k, v in kw.items():
            setattr(q.params, k, v)
        return q

    tv, te, tpe = wl.perturbed_taus((p.tau_v, p.tau_e, p.tau_eps), seed=1212)
    ut, et = fields_fp64(with_tau(tau_v=tv, tau_e=te, tau_eps=tpe))
    z = wl.target_noise(prob.eps.shape, seed=1212).reshape(4, nc)
    ut = ut + 0.01 * np.sqrt((ut ** 2).mean()) * z[:3]
    et = et + 0.01 * np.sqrt((et ** 2).mean()) * z[3]

    def loss(u, e):
        return float(((u - ut) ** 2).sum() + ((e - et) ** 2).sum())

    sim = rlb.from_problems(prob, precision=rlb.FP32, ckpt_every=K, tape_steps=steps)
    fwd_kernel = sim.tune()["name"]  # trial steps leave the state as it was
    stream = sim.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    sim.step(steps)
    ev[1].record(stream)
    m = sim.moments()
    u, e = m["u"].cpu().numpy(), m["eps"].cpu().numpy()
    du = torch.from_numpy(2.0 * (u - ut)).to(sim.device)
    de = torch.from_numpy(2.0 * (e - et)).to(sim.device)
    t0 = time.perf_counter()
    sim.grad(du, de)  # builds and instantiates the reverse sweep's graph
    first_s = time.perf_counter() - t0
    grad_runs = []
    for _ in range(grad_reps):
        torch.cuda.synchronize()
        ev[2].record(stream)
        dtau, de0, du0 = sim.grad(du, de)
        ev[3].record(stream)
        torch.cuda.synchronize()
        grad_runs.append(ev[2].elapsed_time(ev[3]))
    fwd_ms = ev[0].elapsed_time(ev[1])
    grad_ms = float(np.median(grad_runs))
    sim.close()
    h = 1e-4
    fd = []
    for name in ("tau_v", "tau_e", "tau_eps"):
        t0 = getattr(p, name)
        lp = loss(*fields_fp64(with_tau(**{name: t0 + h})))
        lm = loss(*fields_fp64(with_tau(**{name: t0 - h})))
        fd.append((lp - lm) / (2.0 * h))
    fd = np.array(fd)
    scale = max(np.abs(fd).max(), np.abs(dtau).max())
    # the oracle's FP64 adjoint on a small instance of the same generator
    small = wl.shear_vortex(oracle_L, seed=1212)
    rng = np.random.default_rng(6)
    sdu, sde = rng.normal(size=small.u.shape), rng.normal(size=small.eps.shape)
    s2 = rlb.from_problems(small, precision=rlb.FP32, ckpt_every=K, tape_steps=oracle_steps)
    s2.step(oracle_steps)
    g_tau, g_e0, g_u0 = s2.grad(torch.from_numpy(sdu.reshape(3, -1)),
                                torch.from_numpy(sde.reshape(-1)))
    s2.close()
    o_tau, o_e0, o_u0 = oracle.grad(small, oracle_steps, sdu, sde)

    def rel(a, b):
        a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
        return float(np.abs(a - b).max() / np.abs(b).max())

    cell_steps = nc * steps
    total_ms = fwd_ms + grad_ms
    return {"lattice": f"{L}x{L}x1", "steps": steps, "ckpt_every": K,
            "forward_ms": fwd_ms, "forward_kernel": fwd_kernel, "gradient_ms": grad_ms,
            "gradient_ms_runs": [round(x, 4) for x in grad_runs],
            "gradient_first_call_s": first_s,
            "cell_steps_per_s": cell_steps / (total_ms * 1e-3),
            "bytes_per_cell_step": 684,
            "achieved_gbs": 684 * cell_steps / (total_ms * 1e-3) / 1e9,
            "frac": 684 * cell_steps / (total_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "gradient_reverse_gbs": 380 * cell_steps / (grad_ms * 1e-3) / 1e9,
            "graph_launches_per_gradient": 1,
            "loss": loss(u, e), "dL_dtau": [float(x) for x in dtau],
            "dL_dtau_fd": [float(x) for x in fd],
            "error_vs_fd": float(np.abs(dtau - fd).max() / scale),
            "error_vs_oracle_adjoint": {"lattice": f"{oracle_L}x{oracle_L}x1",
                                        "steps": oracle_steps, "dL_dtau": rel(g_tau, o_tau),
                                        "dL_deps0": rel(g_e0.cpu().numpy(), o_e0),
                                        "dL_du0": rel(g_u0.cpu().numpy(), o_u0)}}


def tile_traffic(kernel: str, nx: int, ny: int, cell_bytes: int, corr: int):
    """HBM bytes per cell update of a D2Q9 tile-round kernel on a periodic
    nx x ny lattice: each launch reads every window cell and writes every
    owned cell once and advances H steps. None for other kernels."""
    m = re.match(r"k_d2q9_tiles<\w+,(\d+),(\d+)>/h(\d+)", kernel)
    if not m:
        return None
    tx, ty, h = (int(g) for g in m.groups())
    hx, hy = h, (2 * h if corr else h)
    ox, oy = tx - 2 * hx, ty - 2 * hy
    tiles = -(-nx // ox) * -(-ny // oy)
    read = tiles * tx * ty * cell_bytes
    write = nx * ny * cell_bytes
    return {"window": [tx, ty], "owned": [ox, oy], "steps_per_launch": h,
            "model_bytes_per_cell_update": (read + write) / (nx * ny * h)}


def bench_d2q9(torch, rlb, wl, n: int = 4096, steps: int = 100, warmup: int = 10):
    """The D2Q9 MRT model of Sec. V.A: an n x n periodic random flow in FP32
    and FP64 (one fused launch per step, 2 x 18 populations per cell update),
    also in FP32 with the correction term of Eqs. (37)-(38) (bytes counted at
    the same 144 per cell: the neighbour re-reads are cache hits); the four
    Sec. V.B cases on 4 x 800 as one persistent batch, 400 steps; and the
    corrected moderately relativistic Cases A and D."""
    prob = wl.random_modes(n, n, 1, seed=1211, umax=0.1, amp=0.05, tau_v=0.8, tau_e=0.55,
                           tau_eps=0.7, tau_f=0.8)
    prob.params.lattice = "d2q9"
    cells = prob.params.ncells
    out = {"lattice": f"{n}x{n}x1 periodic", "steps": steps}
    for prec, name, corr in ((rlb.FP32, "fp32", 0), (rlb.FP64, "fp64", 0),
                             (rlb.FP32, "fp32_c7", 1)):
        sim = rlb.from_problems(prob, precision=prec, diag_every=50, correction=corr)
        # 30 trial steps: whole rounds for the tile variants of 2 and 3 steps
        tune = sim.tune(trial_steps=30)
        s0 = sim.sums()
        ms, _ = time_steps(torch, sim, steps, warmup)
        s1 = sim.sums()
        bpc = 2 * 18 * (4 if prec == rlb.FP32 else 8)
        gbs = bpc * cells / (ms * 1e-3) / 1e9
        out[name] = {"ms_per_step": ms, "mlups": cells / (ms * 1e-3) / 1e6,
                     "kernel": tune["name"], "bytes_per_cell": bpc, "achieved_gbs": gbs,
                     "frac": gbs / HBM_PEAK_GBS,
                     "conservation_drift": float(abs(s1 - s0).max() / abs(s0[:2]).max())}
        tiles = tile_traffic(tune["name"], n, n, bpc // 2, corr)
        if tiles:
            # tile rounds move fewer bytes than one step's 2 x 18 values per
            # cell update: achieved_gbs and frac count the round's own HBM
            # traffic, measured by the byte counters when the committed record
            # matches these sources, else the model (window read + owned write
            # per H steps); the bound is the VALU issue rate when the committed
            # VALU record holds this kernel
            meas = measured_d2q9(tune["name"])
            bpu = meas["bytes_per_cell_update"] if meas else tiles["model_bytes_per_cell_update"]
            tiles["hbm_bytes_per_cell_update"] = bpu
            tiles["hbm_bytes_per_cell_update_source"] = "counters" if meas else "model"
            out[name].update({"bytes_per_cell": bpu,
                              "achieved_gbs": bpu * cells / (ms * 1e-3) / 1e9,
                              "frac": bpu * cells / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS})
            out[name]["tile_rounds"] = tiles
            valu = measured_valu(tune["name"])
            if valu:
                rate = valu["valu_per_cell_update"] * cells / (ms * 1e-3) / 1e9
                out[name]["alu_roofline"] = {
                    "bound": "alu", "achieved": rate, "peak": VALU_PEAK_GINST, "unit": "Ginst/s",
                    "frac": rate / VALU_PEAK_GINST,
                    "note": "VALU wave-instructions per cell update (SQ_INSTS_VALU) x cell "
                            "updates per second, against one wave-instruction per CU and cycle"}
        # the timed variant against the oracle: one tile round (3 steps) of the
        # whole lattice
        out[name]["error_vs_oracle"] = live_error(torch, rlb, prob, 3, prec, tune["name"],
                                                  diag_every=50, correction=corr)
        sim.close()
    del prob
    cases = [wl.qgp_tube_2d(c) for c in "ABCD"]
    moderate = [wl.qgp_tube_2d(c, a=1.0 / 30.0, moderate=True, correction=True) for c in "AD"]
    runs = ((rlb.FP64, "cases_A_D_fp64", cases), (rlb.FP32, "cases_A_D_fp32", cases),
            (rlb.FP64, "moderate_A_D_c7_fp64", moderate))
    for prec, name, batch in runs:
        nc = sum(c.params.ncells for c in batch)
        sim = rlb.from_problems(batch, precision=prec)
        tune = sim.tune(trial_steps=50)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.step(400)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out[name] = {"members": " ".join(c.name for c in batch), "steps": 400,
                     "ms_total": ms, "us_per_step": 1e3 * ms / 400,
                     "mlups": nc * 400 / (ms * 1e-3) / 1e6, "kernel": tune["name"],
                     **graph_shape(tune["name"], 400), "inadmissible": sim.moments()["bad"]}
        sim.close()
        out[name]["error_vs_oracle"] = live_error(torch, rlb, batch, 400, prec, tune["name"])
    return out


def bench_eta_s(torch, rlb, wl, n: int = 256, steps: int = 50, warmup: int = 5):
    """The extended model: relaxation times per cell from eta/s (Sec. III.B)
    on the n^3 random flow (FP32), the same lattice under the equation of
    state P = (Gamma - 1)(eps - m n) (Newton recovery), and the Sec. III.B
    tube with its three tau_f choices as one batch, 400 steps (FP64)."""
    prob = wl.random_modes(n, seed=1211, umax=0.1, amp=0.05, tau_v=0.8, tau_e=0.55,
                           tau_eps=0.7, tau_f=0.8)
    prob.params.eta_s, prob.params.a_e, prob.params.a_eps = 0.1, 0.2, 0.5
    sim = rlb.from_problems(prob, precision=rlb.FP32, diag_every=50)
    tune = sim.tune(trial_steps=10)
    ms, _ = time_steps(torch, sim, steps, warmup)
    cells = prob.params.ncells
    gbs = 304 * cells / (ms * 1e-3) / 1e9
    out = {"lattice": f"{n}^3 FP32, eta/s = 0.1", "ms_per_step": ms,
           "mlups": cells / (ms * 1e-3) / 1e6, "kernel": tune["name"], "achieved_gbs": gbs,
           "frac": gbs / HBM_PEAK_GBS}
    sim.close()
    out["error_vs_oracle"] = live_error(torch, rlb, prob, 2, rlb.FP32, tune["name"])
    # the same lattice under P = (Gamma - 1)(eps - m n): Newton recovery per cell
    prob.params.eta_s = 0.0
    prob.params.eos_gamma, prob.params.mass = 1.5, 0.6
    sim = rlb.from_problems(prob, precision=rlb.FP32, diag_every=50)
    tune = sim.tune(trial_steps=10)
    ms, _ = time_steps(torch, sim, steps, warmup)
    gbs = 304 * cells / (ms * 1e-3) / 1e9
    out["general_eos"] = {"eos": "Gamma 1.5, m 0.6", "ms_per_step": ms,
                          "mlups": cells / (ms * 1e-3) / 1e6, "kernel": tune["name"],
                          "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}
    sim.close()
    out["general_eos"]["error_vs_oracle"] = live_error(torch, rlb, prob, 2, rlb.FP32,
                                                       tune["name"])
    del prob
    tubes = [wl.qgp_tube_3d(0.1, tau_f=tf) for tf in ("tau_g", 1.0, 0.6)]
    sim = rlb.from_problems(tubes, precision=rlb.FP64)
    tune = sim.tune(trial_steps=20)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(400)
    e1.record()
    torch.cuda.synchronize()
    out["sec3_tube_batch"] = {"members": "3 x (1x1x800), tau_f = tau_g, 1.0, 0.6", "steps": 400,
                              "ms_total": e0.elapsed_time(e1), "kernel": tune["name"],
                              **graph_shape(tune["name"], 400)}
    sim.close()
    out["sec3_tube_batch"]["error_vs_oracle"] = live_error(torch, rlb, tubes, 400, rlb.FP64,
                                                           tune["name"])
    return out


def cpu_baseline(prob, seconds: float):
    """The FP64 oracle on the host cores, on whole steps of the same lattice.
    Returns the baseline record and the oracle state it reached."""
    import oracle
    threads = oracle.max_threads()
    st = oracle.State.init(prob)
    st.step(1)  # untimed: the first step also pays the first touch of the arrays
    t0 = time.perf_counter()
    st.step(1)
    timed = 1
    dt = time.perf_counter() - t0
    # then whole steps in calls of about 2 s each (a call has a fixed cost of
    # its own) until the time budget is spent
    chunk = max(1, int(2.0 / max(dt, 1e-9)))
    while dt < seconds:
        st.step(chunk)
        timed += chunk
        dt = time.perf_counter() - t0
    cells = prob.params.ncells
    rec = {"value": cells * timed / dt / 1e6, "unit": "MLUPS", "cores": threads,
           "kind": "oracle",
           "sample": f"{timed} FP64 steps of the full {prob.params.nx}x{prob.params.ny}x"
                     f"{prob.params.nz} lattice (after 1 untimed step), {dt:.1f} s"}
    return rec, st, timed + 1


def cpu_baseline_sweep(seconds: float = 4.0) -> dict:
    """The CPU baseline on every benchmark configuration: the FP64 oracle
    (as it stands) timed on all host cores and on one core, in cell updates
    per second (the adjoint: cell-steps of the gradient per second). Each
    figure is a bounded sample of about ``seconds`` of work after one untimed
    step. Context for the GPU figures, not a target."""
    import numpy as np
    import oracle
    import workloads as wl
    cores = oracle.max_threads()

    def timed(run, cells):
        t0 = time.perf_counter()
        run(1)
        one = time.perf_counter() - t0
        n = max(1, int(seconds / max(one, 1e-9)))
        t0 = time.perf_counter()
        run(n)
        dt = time.perf_counter() - t0
        return {"mlups": cells * n / dt / 1e6, "steps": n, "seconds": round(dt, 2)}

    def forward(probs):
        def go(threads):
            oracle.set_threads(threads)
            states = [oracle.State.init(p) for p in probs]

            def run(n):
                for st in states:
                    st.step(n)
            return timed(run, sum(p.params.ncells for p in probs))
        return go

    def adjoint(prob):
        sh = prob.params.shape
        rng = np.random.default_rng(1)
        du, de = rng.standard_normal((3,) + sh), rng.standard_normal(sh)

        def go(threads):
            oracle.set_threads(threads)
            return timed(lambda n: oracle.grad(prob, n, du, de), prob.params.ncells)
        return go

    configs = {
        "shock_tube_1x1x800": forward([wl.shock_tube(800)]),
        "random_modes_256x256x256": forward([wl.random_modes(
            256, seed=1211, umax=0.1, amp=0.05, tau_v=0.8, tau_e=0.55, tau_eps=0.7, tau_f=0.8)]),
        "tube_batch_64": forward(wl.tube_batch()),
        "adjoint_shear_vortex_64x64": adjoint(wl.shear_vortex(64)),
        "blast_128x128x128": forward([wl.blast(128)]),
    }
    out = {"kind": "oracle", "cores": cores, "unit": "MLUPS"}
    try:
        for name, go in configs.items():
            out[name] = {"all_cores": go(cores), "one_core": go(1)}
            log("oracle sweep", name, out[name])
    finally:
        oracle.set_threads(cores)
    return out


def error_vs_oracle(torch, rlb, prob, st, steps: int, kernels, diag_every: int):
    """Max-norm errors of the GPU path against the oracle state of the CPU
    baseline (the same input, the same number of steps), over every cell:
    max|a - b| / max|b| for populations and n, eps; max|a - b| for u. Each GPU
    run uses the kernel variant the benchmark timed for that precision."""
    import numpy as np
    F = st.fields()
    ref = {"f": st.f, "g": st.g, "n": F["n"], "eps": F["eps"], "u": F["u"]}
    out = {"steps": steps, "cells": prob.params.ncells}
    for prec, kernel in kernels:
        sim = rlb.from_problems(prob, precision=prec, diag_every=diag_every)
        sim.variant = sim.variants().index(kernel)
        sim.step(steps)
        f, g = sim.populations()
        m = sim.moments(allow_unphysical=True)
        gpu = {"f": f, "g": g, "n": m["n"], "eps": m["eps"], "u": m["u"]}
        err = {}
        for k, a in gpu.items():
            b = torch.from_numpy(np.ascontiguousarray(ref[k])).to(a.device).reshape(a.shape)
            d = (a - b).abs().max().item()
            err[k] = d if k == "u" else d / b.abs().max().item()
            del b
        err["kernel"] = kernel
        err["inadmissible"] = m["bad"]
        out["fp32" if prec == rlb.FP32 else "fp64"] = err
        del f, g, m, gpu
        sim.close()
    return out


def adjoint_trace(csv_path: str, command: str, grid: str = "512x512x1",
                  steps: int = 1000) -> str:
    """Markdown summary of the reverse sweeps in a rocprofv3 kernel trace of
    the adjoint form: launches and durations of the reverse step (k_adj_step)
    and the recomputation (k_gstep) on one lattice's grid, how many reverse
    steps a recomputation kernel overlapped in time, and per sweep the span
    against the sum of its kernels' durations (a sweep: `steps` consecutive
    reverse steps, one gradient of a run of that many steps)."""
    import csv
    import statistics

    rows = []
    for r in csv.DictReader(open(csv_path)):
        name = r["Kernel_Name"]
        kind = "adj" if "k_adj_step" in name else ("g" if "k_gstep" in name else None)
        if kind is None or "x".join(r[f"Grid_Size_{a}"] for a in "XYZ") != grid:
            continue
        rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), kind))
    rows.sort()
    adj = [(s, e) for s, e, k in rows if k == "adj"]
    rec = [(s, e) for s, e, k in rows if k == "g"]
    out = [f"Command: `{command}`", ""]
    if not adj:
        return "\n".join(out + [f"No reverse steps on the {grid} grid.", ""])
    # sweeps (one per gradient): consecutive runs of `steps` reverse steps
    sweeps = [adj[i:i + steps] for i in range(0, len(adj), steps)]
    overlapped, j = 0, 0
    for s, e in adj:
        while j < len(rec) and rec[j][1] < s:
            j += 1
        k = j
        while k < len(rec) and rec[k][0] < e:
            if rec[k][1] > s:
                overlapped += 1
                break
            k += 1

    def stat(v):
        us = [(e - s) / 1e3 for s, e in v]
        return len(us), statistics.mean(us), statistics.median(us)

    na, ma, da = stat(adj)
    ng, mg, dg = stat(rec) if rec else (0, 0.0, 0.0)
    out += [f"Kernels on the {grid} grid:", "",
            "| kernel | launches | mean (us) | median (us) |", "|---|---|---|---|",
            f"| `k_adj_step` (reverse step) | {na} | {ma:.2f} | {da:.2f} |",
            f"| `k_gstep` (recomputation) | {ng} | {mg:.2f} | {dg:.2f} |", "",
            f"Reverse steps overlapped in time by a recomputation kernel: {overlapped} of {na} "
            f"({100.0 * overlapped / na:.1f} %).", "",
            "| sweep | reverse steps | span (ms) | reverse-step time (ms) | recomputation time "
            "within the span (ms) | span / sum of both |", "|---|---|---|---|---|---|"]
    for i, sw in enumerate(sweeps):
        s0, s1 = sw[0][0], sw[-1][1]
        ta = sum(e - s for s, e in sw) / 1e6
        tg = sum(min(e, s1) - max(s, s0) for s, e in rec if e > s0 and s < s1) / 1e6
        span = (s1 - s0) / 1e6
        out.append(f"| {i} | {len(sw)} | {span:.2f} | {ta:.2f} | {tg:.2f} | "
                   f"{span / (ta + tg):.2f} |")
    return "\n".join(out) + "\n"


def adjoint_traffic(fetch_csv: str, write_csv: str, command: str, cells: int = 512 * 512) -> str:
    """Markdown table of the HBM bytes per dispatch of the reverse-sweep
    kernels on a lattice of `cells` cells (one thread per cell), from one
    FETCH_SIZE and one WRITE_SIZE rocprofv3 --pmc run of the adjoint form with
    --copy-calibration: each counter scaled by what it reads for the 1 GiB
    copy in the same run, set against the algorithmic bytes (reverse step:
    19 taped populations and 19 adjoint populations read, 19 written, 228 B
    per cell in FP32; recomputation: 19 read, 19 written, 152 B)."""
    import collections
    import csv

    def short(name):
        name = name.replace("(anonymous namespace)::", "").replace("void ", "")
        return re.sub(r"^.*::(?=k_)", "", name.split("(")[0])

    vals = collections.defaultdict(list)
    copy = {}
    for path in (fetch_csv, write_csv):
        for r in csv.DictReader(open(path)):
            k, g, c = r["Kernel_Name"], int(r["Grid_Size"]), r["Counter_Name"]
            v = float(r["Counter_Value"]) * 1024.0
            if "copyBuffer" in k:
                copy.setdefault(c, []).append(v)
            elif g == cells and short(k).startswith(("k_adj_step", "k_gstep")):
                vals[(short(k), c)].append(v)
    # the 1 GiB copy: the largest copy dispatches (the tape's checkpoints are
    # copies of one state, far smaller)
    big = {c: [x for x in v if x > 0.5 * max(v)] for c, v in copy.items()}
    scale = {c: (1 << 30) / (sum(v) / len(v)) for c, v in big.items()}
    out = [f"Command: `{command}`", "",
           f"Copy calibration (1 GiB): FETCH_SIZE x {scale.get('FETCH_SIZE', float('nan')):.4f}, "
           f"WRITE_SIZE x {scale.get('WRITE_SIZE', float('nan')):.4f}.", "",
           "| kernel | dispatches | fetch B / dispatch | write B / dispatch | total / algorithmic |",
           "|---|---|---|---|---|"]
    for name in sorted({k for k, _ in vals}):
        f, w = vals.get((name, "FETCH_SIZE")), vals.get((name, "WRITE_SIZE"))
        if not f or not w or "FETCH_SIZE" not in scale or "WRITE_SIZE" not in scale:
            continue
        esz = 8 if "double" in name else 4
        alg = (57 if name.startswith("k_adj_step") else 38) * esz * cells
        fb = sum(f) / len(f) * scale["FETCH_SIZE"]
        wb = sum(w) / len(w) * scale["WRITE_SIZE"]
        out.append(f"| `{name}` | {len(f)} | {fb:.4e} | {wb:.4e} | {(fb + wb) / alg:.4f} |")
    return "\n".join(out) + "\n"


def summarize_trace(csv_path: str, command: str, top: int = 25, min_launches: int = 40) -> str:
    """Markdown tables of a rocprofv3 --kernel-trace --stats run: the
    kernel_stats.csv summary, and (from the kernel_trace.csv beside it) the
    step kernels split by launch grid, since one kernel serves several
    workloads in the default run."""
    import collections
    import csv
    import os

    def short(name):
        name = name.replace("rlb::(anonymous namespace)::", "").replace("void ", "")
        return name.split("(")[0]

    rows = list(csv.DictReader(open(csv_path)))
    out = [f"Command: `{command}`", "",
           f"The {top} kernels with the most total time:", "",
           "| kernel | calls | average (us) | min (us) | max (us) | total (ms) | % |",
           "|---|---|---|---|---|---|---|"]
    rest = rows[top:]
    rows = rows[:top]
    for r in rows:
        out.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    if rest:
        out.append(f"| {len(rest)} more kernels | {sum(int(r['Calls']) for r in rest)} | | | | "
                   f"{sum(float(r['TotalDurationNs']) for r in rest) / 1e6:.2f} | "
                   f"{sum(float(r['Percentage']) for r in rest):.1f} |")
    trace = csv_path.replace("kernel_stats.csv", "kernel_trace.csv")
    if trace != csv_path and os.path.exists(trace):
        groups = collections.defaultdict(list)
        for r in csv.DictReader(open(trace)):
            name = short(r["Kernel_Name"])
            if not name.startswith(("k_step", "k_adj_step", "k_gstep", "k_d2q9_lattice", "k_d2q9_members")):
                continue
            grid = "x".join(r[f"Grid_Size_{a}"] for a in "XYZ")
            block = "x".join(r[f"Workgroup_Size_{a}"] for a in "XYZ")
            groups[(name, grid, block)].append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        out += ["", f"Step kernels by launch grid (threads), from the kernel_trace.csv of the same "
                f"run ({min_launches} or more launches):", "",
                "| kernel | grid | block | launches | average (us) | min (us) | max (us) |",
                "|---|---|---|---|---|---|---|"]
        for (name, grid, block), d in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
            if len(d) < min_launches:
                continue
            out.append(f"| `{name}` | {grid} | {block} | {len(d)} | {sum(d) / len(d):.1f} | "
                       f"{min(d):.1f} | {max(d):.1f} |")
    return "\n".join(out) + "\n"


def write_traffic(*csvs: str, cells: int = 256 ** 3) -> dict:
    """HBM bytes per dispatch of every step-kernel variant from pairs of PMC
    runs (FETCH_SIZE, WRITE_SIZE in KiB; e.g. one pair per precision), each
    counter scaled by what it reads for the 1 GiB plain copy of
    --copy-calibration in the same run."""
    if len(csvs) < 2 or len(csvs) % 2:
        raise ValueError("write_traffic takes FETCH_SIZE / WRITE_SIZE csv pairs")
    out = {}
    for i in range(0, len(csvs), 2):
        rec = _traffic_pair(csvs[i], csvs[i + 1], cells)
        out["_calibration" + ("" if i == 0 else f"_run{i // 2}")] = rec.pop("_calibration")
        out.update(rec)
    return out


def _traffic_pair(fetch_csv: str, write_csv: str, cells: int) -> dict:
    import collections
    import csv
    vals = collections.defaultdict(list)
    for path in (fetch_csv, write_csv):
        for r in csv.DictReader(open(path)):
            vals[(r["Kernel_Name"], r["Grid_Size"], r["Counter_Name"])].append(
                float(r["Counter_Value"]) * 1024.0)
    copy = {c: sum(v) / len(v) for (k, g, c), v in vals.items()
            if "copyBuffer" in k and g == "131072"}
    scale = {c: (1 << 30) / copy[c] for c in copy}
    out = {"_calibration": {"copy_bytes": 1 << 30, "counter_bytes": copy, "scale": scale}}
    for (k, g, c), v in vals.items():
        # k_step_lattice<T, BX, BY, CZ, DIAG, EXT, NTS>: the launches with fused
        # diagnostics and the eta/s kernels are not priced
        m = re.search(r"k_step_lattice<(\w+), (\d+), (\d+), (\d+), (\w+), (\w+), (\w+)>", k)
        if not m or m.group(5) == "true" or m.group(6) == "true":
            continue
        name = "k_step_lattice<{},{},{},{}>".format(*m.groups()[:4])
        rec = out.setdefault(name, {"cells": cells, "source_hash": kernel_hash()})
        rec[c.lower() + "_bytes"] = sum(v) / len(v) * scale[c]
    for name, rec in out.items():
        if name.startswith("_") or "fetch_size_bytes" not in rec or "write_size_bytes" not in rec:
            continue
        esz = 4 if "float" in name else 8
        rec["bytes_per_launch"] = rec["fetch_size_bytes"] + rec["write_size_bytes"]
        rec["algorithmic_bytes"] = 2 * 38 * esz * cells
        rec["ratio"] = rec["bytes_per_launch"] / rec["algorithmic_bytes"]
    return out


# MI355X: 256 CUs of 4 SIMDs; a SIMD takes 4 cycles per wave64 VALU
# instruction, so a CU issues at most one wave-level VALU instruction a cycle.
CU_NUM = 256
XCC_NUM = 8


def valu_summary(csv_path: str, command: str) -> str:
    """Markdown table of the VALU load of the step kernels from one rocprofv3
    --pmc run of SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU, SQ_INSTS_LDS, SQ_WAVES
    and GRBM_GUI_ACTIVE: per kernel and launch grid, the mean over its
    dispatches of the duration (the dispatch timestamps), the shader clock
    (GRBM_GUI_ACTIVE, summed over the 8 XCDs, per XCD and second), the
    issue fraction (wave-level VALU instructions over one per CU and cycle)
    and the VALU busy fraction (SQ_ACTIVE_INST_VALU quad-cycles summed over
    the SIMDs, over CUs x cycles, as rocprofv3's VALUBusy). For launches of
    a few tens of microseconds GRBM_GUI_ACTIVE also counts cycles around the
    kernel (the clock column then reads above 2.4 GHz) and both fractions
    read low; the last fraction counts the cycles of the dispatch's own
    duration at 2.4 GHz instead."""
    import collections
    import csv

    def short(name):
        name = name.replace("rlb::(anonymous namespace)::", "").replace("void ", "")
        return name.split("(")[0]

    groups = collections.defaultdict(lambda: collections.defaultdict(list))
    dur = collections.defaultdict(dict)
    for r in csv.DictReader(open(csv_path)):
        name = short(r["Kernel_Name"])
        if not name.startswith(("k_step", "k_d2q9", "k_adj_step", "k_gstep")):
            continue
        key = (name, int(r["Grid_Size"]), int(r["Workgroup_Size"]))
        groups[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
        dur[key][r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    out = [f"Command: `{command}`", "",
           "| kernel | grid (threads) | block | dispatches | average (us) | clock (GHz) | "
           "VALU wave-instructions per dispatch | issue fraction | VALU busy | LDS / VALU | "
           "issue fraction at 2.4 GHz |",
           "|---|---|---|---|---|---|---|---|---|---|---|"]
    need = ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_LDS", "GRBM_GUI_ACTIVE")
    rows = []
    for key, c in groups.items():
        if any(n not in c for n in need):
            continue
        mean = {n: sum(v) / len(v) for n, v in c.items()}
        t = sum(dur[key].values()) / len(dur[key])
        cycles = mean["GRBM_GUI_ACTIVE"] / XCC_NUM
        rows.append((key, len(dur[key]), t, cycles / t / 1e9, mean["SQ_INSTS_VALU"],
                     mean["SQ_INSTS_VALU"] / (CU_NUM * cycles),
                     mean["SQ_ACTIVE_INST_VALU"] / (CU_NUM * cycles),
                     mean["SQ_INSTS_LDS"] / max(mean["SQ_INSTS_VALU"], 1.0),
                     mean["SQ_INSTS_VALU"] / (CU_NUM * t * 2.4e9)))
    for (name, grid, block), n, t, ghz, valu, issue, busy, lds, nominal in sorted(
            rows, key=lambda r: -r[1] * r[2]):
        out.append(f"| `{name}` | {grid} | {block} | {n} | {t * 1e6:.1f} | {ghz:.2f} | "
                   f"{valu:.4g} | {issue:.3f} | {busy:.3f} | {lds:.3f} | {nominal:.3f} |")
    return "\n".join(out) + "\n"


def d2q9_kernel_name(kernel: str, grid: int, n: int = 4096):
    """(variant name, steps per launch) of a D2Q9 lattice-path dispatch on the
    n x n periodic lattice, from the mangled-template name in a rocprofv3
    record and its grid (threads): k_d2q9_lattice<T, BX, BY, CY, DIAG, CORR,
    EXT, NTS>, k_d2q9_lattice_c7<T, BX, BY, DIAG, EXT, NTS> (one step a
    launch) and k_d2q9_tiles<T, TX, TY, NTH, CORR, EXT> (H steps a launch,
    H recovered from the number of tiles in the grid). None for launches
    with fused diagnostics, the extended model, or other kernels."""
    m = re.search(r"k_d2q9_tiles<(\w+), (\d+), (\d+), (\d+), (\w+), (\w+)", kernel)
    if m:
        typ, tx, ty, nth, corr, ext = m.groups()
        if ext == "true":
            return None
        tx, ty, nth = int(tx), int(ty), int(nth)
        tiles = grid // nth
        c = corr == "true"
        H = next((h for h in range(1, 9)
                  if -(-n // (tx - 2 * h)) * -(-n // (ty - 2 * (2 * h if c else h))) == tiles),
                 None)
        if H is None:
            return None
        return f"k_d2q9_tiles<{typ},{tx},{ty}>/h{H}" + ("+c7" if c else ""), H
    m = re.search(r"k_d2q9_lattice<(\w+), (\d+), (\d+), (\d+), (\w+), (\w+), (\w+)", kernel)
    if m:
        typ, bx, by, cy, diag, corr, ext = m.groups()
        if diag == "true" or ext == "true":
            return None
        return f"k_d2q9_lattice<{typ},{bx},{by},{cy}>" + ("+c7" if corr == "true" else ""), 1
    m = re.search(r"k_d2q9_lattice_c7<(\w+), (\d+), (\d+), (\w+), (\w+)", kernel)
    if m:
        typ, bx, by, diag, ext = m.groups()
        if diag == "true" or ext == "true":
            return None
        return f"k_d2q9_lattice<{typ},{bx},{by},1>+c7", 1
    return None


def d2q9_traffic(fetch_csv: str, write_csv: str, n: int = 4096) -> dict:
    """HBM bytes of the D2Q9 lattice-path kernels on the n x n lattice from two
    PMC runs (FETCH_SIZE, WRITE_SIZE), scaled as in write_traffic: per launch,
    and per cell update (a tile-round launch advances H steps), against the
    one-step 2 x 18 values per cell."""
    import collections
    import csv
    vals = collections.defaultdict(list)
    for path in (fetch_csv, write_csv):
        for r in csv.DictReader(open(path)):
            vals[(r["Kernel_Name"], int(r["Grid_Size"]), r["Counter_Name"])].append(
                float(r["Counter_Value"]) * 1024.0)
    copy = {c: sum(v) / len(v) for (k, g, c), v in vals.items()
            if "copyBuffer" in k and g == 131072}
    scale = {c: (1 << 30) / copy[c] for c in copy}
    recs = collections.defaultdict(dict)
    for (k, g, c), v in vals.items():
        nm = d2q9_kernel_name(k, g, n)
        if nm:
            recs[nm][c] = sum(v) / len(v) * scale[c]
    cells = n * n
    out = {"lattice": f"{n}x{n}", "calibration": scale, "source_hash": kernel_hash(D2Q9_SOURCES),
           "kernels": {}}
    for (name, H), r in sorted(recs.items()):
        if "FETCH_SIZE" not in r or "WRITE_SIZE" not in r:
            continue
        esz = 4 if "float" in name else 8
        total = r["FETCH_SIZE"] + r["WRITE_SIZE"]
        out["kernels"][name] = {"bytes_per_launch": total, "steps_per_launch": H,
                                "bytes_per_cell_update": total / (cells * H),
                                "one_step_bytes_per_cell_update": 2 * 18 * esz,
                                "ratio_to_one_step": total / (cells * H) / (2 * 18 * esz)}
    return out


def valu_record(csv_path: str, n: int = 4096) -> dict:
    """VALU wave-instructions per cell update of the D2Q9 lattice-path kernels
    on the n x n lattice, from the same PMC run as valu_summary."""
    import collections
    import csv
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] != "SQ_INSTS_VALU":
            continue
        nm = d2q9_kernel_name(r["Kernel_Name"], int(r["Grid_Size"]), n)
        if nm:
            vals[nm].append(float(r["Counter_Value"]))
    out = {"lattice": f"{n}x{n}", "source_hash": kernel_hash(D2Q9_SOURCES), "kernels": {}}
    for (name, H), v in sorted(vals.items()):
        out["kernels"][name] = {"valu_per_launch": sum(v) / len(v), "steps_per_launch": H,
                                "valu_per_cell_update": sum(v) / len(v) / (n * n * H)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the 256^3 run is 500 steps: 50 untimed, then 450 timed
    ap.add_argument("--steps", type=int, default=450)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--oracle-sweep", action="store_true",
                    help="time the CPU oracle on every configuration (all cores and one "
                         "core), print one JSON line and exit")
    ap.add_argument("--no-forms", action="store_true", help="only the headline FP32 step")
    ap.add_argument("--forms", default="",
                    help="comma list of the forms to run besides the headline (default: all): "
                         "fp64, shock_tube, batched, adjoint, blast_512, d2q9, eta_s, "
                         "copy_ceiling")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--diag-every", type=int, default=50,
                    help="fuse the FP64 conservation sums into every N-th step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for HBM byte counters)")
    ap.add_argument("--adjoint-trace", nargs=2, metavar=("TRACE_CSV", "COMMAND"),
                    help="summarise the reverse sweeps in a rocprofv3 kernel_trace.csv")
    ap.add_argument("--adjoint-traffic", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "COMMAND"),
                    help="print the HBM bytes per dispatch of the reverse-sweep kernels from two "
                         "PMC runs of the adjoint form and exit")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("CSV", "COMMAND"),
                    help="print a markdown summary of a rocprofv3 kernel_stats.csv and exit")
    ap.add_argument("--valu-summary", nargs=2, metavar=("CSV", "COMMAND"),
                    help="print the VALU load of the step kernels from one PMC run (and write "
                         "profiles/valu_d2q9.json for the D2Q9 kernels it holds) and exit")
    ap.add_argument("--d2q9-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_d2q9.json (HBM bytes of the D2Q9 kernels) from "
                         "two PMC runs and exit")
    ap.add_argument("--write-traffic", nargs="+", metavar="CSV",
                    help="write profiles/traffic.json from FETCH_SIZE / WRITE_SIZE csv pairs "
                         "(one pair per PMC run pair) and exit")
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_trace(*args.summarize_trace), end="")
        return
    if args.adjoint_trace:
        print(adjoint_trace(*args.adjoint_trace), end="")
        return
    if args.adjoint_traffic:
        print(adjoint_traffic(*args.adjoint_traffic), end="")
        return
    if args.oracle_sweep:
        print(json.dumps(cpu_baseline_sweep()), flush=True)
        return
    if args.d2q9_traffic:
        rec = d2q9_traffic(*args.d2q9_traffic)
        with open(D2Q9_TRAFFIC_FILE, "w") as fh:
            json.dump(rec, fh, indent=1, sort_keys=True)
        print(json.dumps(rec, indent=1, sort_keys=True))
        return
    if args.valu_summary:
        print(valu_summary(*args.valu_summary), end="")
        rec = valu_record(args.valu_summary[0])
        if rec["kernels"]:
            with open(VALU_FILE, "w") as fh:
                json.dump(rec, fh, indent=1, sort_keys=True)
        return
    if args.write_traffic:
        rec = write_traffic(*args.write_traffic)
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(rec, fh, indent=1, sort_keys=True)
        print(json.dumps(rec, indent=1, sort_keys=True))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "slab decomposition is a design only; this library runs on one GPU", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1211_3286_amd as rlb
    import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    prec = rlb.FP32 if args.precision == "fp32" else rlb.FP64
    log(f"lattice {args.size}^3 {args.precision}: warmup {args.warmup}, steps {args.steps}")
    head = bench_lattice(torch, rlb, wl, args.size, prec, args.steps, args.warmup,
                         args.diag_every)
    log("headline", {k: v for k, v in head.items() if k not in ("problem", "variant_ms")})
    traffic = measured_traffic(head["kernel"], head["cells"])
    roof = {"bound": "hbm", "achieved": round(head["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(head["frac"], 4), "traffic": traffic,
            "kernel": head["kernel"], "algorithmic_bytes_per_launch":
                head["bytes_per_cell"] * head["cells"]}
    forms = {}
    sel = set(args.forms.split(",")) if args.forms else None

    def want(name):
        return not args.no_forms and (sel is None or name in sel)

    other = rlb.FP64 if prec == rlb.FP32 else rlb.FP32
    oname = "fp64" if other == rlb.FP64 else "fp32"
    if want(oname):
        o = bench_lattice(torch, rlb, wl, args.size, other, max(args.steps // 2, 10),
                          max(args.warmup // 2, 2), args.diag_every)
        forms[oname] = {k: o[k] for k in ("mlups", "ms_per_step", "achieved_gbs", "frac",
                                          "kernel", "conservation_drift")}
        forms[oname]["traffic"] = measured_traffic(o["kernel"], o["cells"])
        log("other precision", forms)
    runs = (("shock_tube", bench_shock_tube), ("batched", bench_batched),
            ("adjoint", bench_adjoint), ("blast_512", bench_blast), ("d2q9", bench_d2q9),
            ("eta_s", bench_eta_s))
    for name, fn in runs:
        if want(name):
            forms[name] = fn(torch, rlb, wl)
            log(name, forms[name])
    if want("copy_ceiling"):
        # the runtime's own device-to-device copy of the bytes one FP32 step
        # moves (38 x 4 B per cell read, the same written), as context for the
        # step's rate: step_speed_over_copy is a ratio of speeds, not a
        # fraction of a peak (the fused step moves its bytes faster than it)
        cc = copy_calibration(torch, nbytes=38 * 4 * head["cells"], reps=20)
        cc["step_speed_over_copy"] = head["achieved_gbs"] / cc["gbs"]
        forms["copy_ceiling"] = cc
        log("copy ceiling", cc)
    if args.copy_calibration:
        forms["copy_calibration"] = copy_calibration(torch)
        log("copy", forms["copy_calibration"])
    cpu = errors = None
    if not args.no_cpu:
        log("cpu baseline ...")
        cpu, ost, osteps = cpu_baseline(head["problem"], args.cpu_seconds)
        log("cpu", cpu)
        kernels = [(prec, head["kernel"])]
        if not args.no_forms:
            kernels.append((other, forms["fp64" if other == rlb.FP64 else "fp32"]["kernel"]))
        errors = error_vs_oracle(torch, rlb, head["problem"], ost, osteps, kernels,
                                 args.diag_every)
        log("error vs oracle", errors)
        del ost
    p = head["problem"].params
    line = {
        "metric": METRIC, "value": round(head["mlups"], 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == rlb.FP32 else "f64", "data": "synthetic",
        "config": {"workload": f"random_modes_{p.nx}x{p.ny}x{p.nz}_periodic_seed1211",
                   "lattice": "D3Q19 f+g", "cells": head["cells"], "tau_v": p.tau_v,
                   "tau_e": p.tau_e, "tau_eps": p.tau_eps, "tau_f": p.tau_f,
                   "recovery": "fp64", "diag_every": args.diag_every},
        "roofline": roof, "cpu_baseline": cpu, "error_vs_oracle": errors,
        "conservation_drift": head["conservation_drift"], "inadmissible": head["inadmissible"],
        "forms": forms,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
