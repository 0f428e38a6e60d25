"""Throughput benchmark of the split-form DGSEM hot path on one MI355X.

Default workload: Taylor-Green vortex, Ma 0.1, Re 1600, Pr 0.72, N = 7 on
64^3 periodic elements (134 M nodes), Pirozzoli split flux + Roe, BR1
lifting (split: one lifting launch per step), FP64, LSERK4: the configuration
the metric is quoted on (FP64
against the mixed-precision operator at its stated error; the adjoint of
the N = 5, 16^3 TGV beside it).  A "step" is one Runge-Kutta step (5 stages) over the
whole mesh.  The metric is DOF-stage updates per second (1/PID with the GPU as
the single "core"; DOF counts nodes).  Inputs are resident in HBM before the
timed region; the timed region is bracketed by torch.cuda.synchronize().

Prints one JSON line with the throughput, the roofline of the dominant kernel
(measured with HIP events on the library's stream during the timed region:
160 B per DOF and launch -- read U and the register, write the register and U
-- over the average launch time, against 8 TB/s), its FP64 FLOP rate (the
kernel's flops per DOF, counted with rocprofv3, over the same time, against
78.6 TFLOP/s), and the CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-stage updates/s (1/PID) FP64 vs mixed at stated err; adjoint/forward time"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

WORKLOADS = {
    # name: (N, nelem, equations, vol_flux, surf_flux, mu, blending, description)
    "tgv_n5_32": (5, (32, 32, 32), 1, 1, 1, 1.0 / 1600, 0,
                  "TGV Ma0.1 Re1600 Pr0.72, N=5, 32^3 elems, PI+Roe, BR1, LSERK4"),
    "tgv_n7_64": (7, (64, 64, 64), 1, 1, 1, 1.0 / 1600, 0,
                  "TGV Ma0.1 Re1600 Pr0.72, N=7, 64^3 elems, PI+Roe, BR1, LSERK4"),
    "density_wave_n3_4": (3, (4, 4, 4), 0, 0, 0, 0.0, 0,
                          "Euler density wave, N=3, 4^3 elems, KG+LLF, LSERK4"),
    "freestream_euler_n7_64": (7, (64, 64, 64), 0, 0, 0, 0.0, 0,
                               "Euler freestream Ma0.5, N=7, 64^3 elems, KG+LLF, LSERK4"),
    "freestream_ns_n7_64": (7, (64, 64, 64), 1, 1, 1, 1.0 / 1600, 0,
                            "NS freestream Ma0.5, N=7, 64^3 elems, PI+Roe, BR1, LSERK4"),
    "sod_n5_64x8x8": (5, (64, 8, 8), 0, 0, 0, 0.0, 1,
                      "Euler Sod tube, N=5, 64x8x8 elems, KG+LLF, DG/FV blending (minmod), LSERK4"),
    "sod_ns_n4_256x16x16": (4, (256, 16, 16), 1, 0, 0, 2e-6, 1,
                            "High-Reynolds viscous Sod tube (Navier-Stokes, mu 2e-6, Pr 0.72), N=4, 256x16x16 elems, "
                            "KG+LLF, DG/FV blending of the advective terms (minmod), BR1, LSERK4"),
    "tgv_les_n5_32": (5, (32, 32, 32), 1, 1, 1, 1.0 / 1600, 0,
                      "TGV Ma0.1 Re1600 LES (Smagorinsky C_s=0.17, Pr_t=0.9), N=5, 32^3 elems, PI+Roe, BR1, "
                      "LSERK4"),
    "tgv_curved_n5_32": (5, (32, 32, 32), 1, 1, 1, 1.0 / 1600, 0,
                         "TGV Ma0.1 Re1600 Pr0.72 on a warped periodic mesh (curved elements, curl-form metric "
                         "terms, displacement amplitude 0.04 of the box), N=5, 32^3 elems, PI+Roe, BR1, LSERK4"),
    "channel_wm_n5_32": (5, (32, 32, 32), 1, 1, 1, 2e-5, 0,
                         "Wall-modelled channel LES, 2pi x 2 x pi, walls normal to y (Spalding's law with van Driest "
                         "transformation, u_inf 1, Ma_inf 0.7), Smagorinsky C_s=0.17, centre-line Ma 0.7, "
                         "mu 2e-5, N=5, 32^3 elems, PI+Roe, BR1, LSERK4"),
}

# Wall-modelled workloads: (wall direction, u_inf, Ma_inf of the van Driest
# transformation).
WALLS = {"channel_wm_n5_32": (1, 1.0, 0.7)}

# Curved workloads: amplitude of the smooth periodic node displacement
# (inputs.warped_coordinates); the stage kernel then also reads the metric
# terms, 10 doubles = 80 B per node and launch.
CURVED = {"tgv_curved_n5_32": 0.04}
METRIC_BYTES_PER_NODE = 80.0

# Smagorinsky coefficient of the LES workloads (standard model, constant C_s).
MODEL_CS = {"tgv_les_n5_32": 0.17, "channel_wm_n5_32": 0.17}


# Element counts of the freestream size sweep: 2^15 ... 2^21 elements, grown
# one direction at a time (z, then y, then x) from 32^3.
SWEEP_MESHES = [(32, 32, 32), (32, 32, 64), (32, 64, 64), (64, 64, 64), (64, 64, 128), (64, 128, 128),
                (128, 128, 128)]


def curved_nodes(name, N, nelem):
    from paper_2306_12891_amd import inputs
    return inputs.warped_coordinates(N, nelem, amp=CURVED[name]) if name in CURVED else None


def initial_state(name, N, nelem):
    from paper_2306_12891_amd import inputs
    if name.startswith("tgv"):
        return inputs.tgv(N, nelem, xnodes=curved_nodes(name, N, nelem))
    if name.startswith("density_wave"):
        return inputs.density_wave(N, nelem)
    if name.startswith("freestream"):
        return inputs.freestream(N, nelem)
    if name.startswith("sod"):
        return inputs.sod(N, nelem, (0, 0, 0), (1.0, 0.125, 0.125))
    if name.startswith("channel"):
        return inputs.channel(N, nelem, *domain(name))
    raise KeyError(name)


def domain(name):
    if name.startswith("sod"):
        return (0.0, 0.0, 0.0), (1.0, 0.125, 0.125)
    if name.startswith("channel"):
        return (0.0, 0.0, 0.0), (2 * math.pi, 2.0, math.pi)
    return (0.0, 0.0, 0.0), (2 * math.pi,) * 3


# HBM bytes per launch of the stage kernel measured with rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE (separate runs), each scaled by the plain-copy
# calibration (FETCH x 2.000, WRITE x 1.000); averages over the five stage
# launches of one step (the TGV workloads with the split lifting); see
# profiles/k_stage_*.md.
# Valid only for the kernel source they were taken on (sha256 prefix).
MEASURED_TRAFFIC = {
    "kernel_sha": "cc42175a04ddafbd",
    "tgv_n7_64": {"bytes_per_launch": 26891.8e6, "fetch": 14651.1e6, "write": 12240.7e6},
    "tgv_n5_32": {"bytes_per_launch": 1599.7e6, "fetch": 874.4e6, "write": 725.3e6},
    "freestream_euler_n7_64": {"bytes_per_launch": 20721.4e6, "fetch": 11057.7e6, "write": 9663.7e6},
    "tgv_curved_n5_32": {"bytes_per_launch": 2056.2e6, "fetch": 1521.0e6, "write": 535.2e6},
    "channel_wm_n5_32": {"bytes_per_launch": 1389.6e6, "fetch": 864.3e6, "write": 525.3e6},
    "sod_ns_n4_256x16x16": {"bytes_per_launch": 2302.3e6, "fetch": 1675.6e6, "write": 626.7e6},
    "tgv_les_n5_32": {"bytes_per_launch": 1398.8e6, "fetch": 872.3e6, "write": 526.5e6},
}


# FP64 (mixed: FP32) floating-point operations of the stage kernel per DOF
# and launch, counted with rocprofv3 (SQ_INSTS_VALU_FMA_F64 x 2 + ADD + MUL +
# TRANS, times 64 lanes, over the DOF of the launch; averages over the five
# stage launches of one step; profiles/k_stage_*.md); valid only for the
# kernel source they were counted on (sha256 prefix).
KERNEL_FLOPS = {
    "kernel_sha": "cc42175a04ddafbd",
    "tgv_n7_64": {"stage_flops_per_dof": 1418.5},
    "tgv_n5_32": {"stage_flops_per_dof": 1583.6},
    "freestream_euler_n7_64": {"stage_flops_per_dof": 717.2},
    "tgv_curved_n5_32": {"stage_flops_per_dof": 2062.5},
    "channel_wm_n5_32": {"stage_flops_per_dof": 1416.3},
    "sod_ns_n4_256x16x16": {"stage_flops_per_dof": 1068.3},
    "tgv_les_n5_32": {"stage_flops_per_dof": 1403.3},
}


def kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("dg_kernels.hip", "dg_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2306_12891_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stage_bytes_per_step(nodes):
    """Algorithmic HBM bytes of the stage kernel over the five stages of one
    step: read U (40 B/node) and write U (40); the register G is written in
    stages 1-4 and read in stages 2-5 (stage 1 has A_1 = 0, the stage-5
    register is dead): 2 x 120 + 3 x 160 = 720 B per node."""
    return 720.0 * nodes


def adjoint_leg(torch, dg, inputs, steps=200, every=20, n_dirs=8, eps=1e-6):
    """Gradient of the volume-averaged kinetic energy after `steps` LSERK4
    steps of the TGV (N = 5, 16^3 elements, symmetry-broken start) with respect
    to the initial state, by the checkpointed reverse rollout; timed against
    the forward rollout and checked against central differences."""
    N, nelem, mu = 5, (16, 16, 16), 1.0 / 1600
    op = dg.DG(nelem, N, gamma=1.4, mu=mu, equations=dg.NS, vol_flux=dg.PI, surf_flux=dg.ROE, Pr=0.72)
    U0 = torch.from_numpy(inputs.tgv(N, nelem, symmetry_break=True)).to("cuda:0")
    W = op.node_weights("cuda:0")
    vol = (2 * math.pi) ** 3
    dt = op.max_dt(U0, 0.5)

    def ke(U):
        m = U[:, 1:4]
        return torch.sum(W * 0.5 * torch.sum(m * m, 1) / U[:, 0]) / vol

    def forward(U):
        V = U.clone()
        op.rk_steps(V, dt, steps)
        return ke(V).item()

    forward(U0)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    forward(U0)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    # warm-up of the gradient (its stage-state record is a 3.5 GB allocation
    # that the timed run then takes from torch's cache), as for the forward
    xw = U0.clone().requires_grad_(True)
    ke(dg.rollout(op, xw, dt, steps, checkpoint_every=every)).backward()
    del xw
    x = U0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ke(dg.rollout(op, x, dt, steps, checkpoint_every=every)).backward()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    g = x.grad.detach()
    errs = []
    for k in range(n_dirs):
        v = torch.from_numpy(inputs.random_directions(tuple(U0.shape), k)).to("cuda:0")
        fd = (forward(U0 + eps * v) - forward(U0 - eps * v)) / (2 * eps)
        ad = torch.sum(g * v).item()
        errs.append(abs(fd - ad) / abs(ad))
    # single-operator timing: dg_vjp against dg_time_derivative
    lam = torch.from_numpy(inputs.random_directions(tuple(U0.shape), 99)).to("cuda:0")
    op.set_profiling(True)
    for _ in range(10):
        op.time_derivative(U0)
        op.vjp(U0, lam)
    prof = op.profile_read()
    op.set_profiling(False)
    t_op = prof["stage"][0] + prof["lift"][0]
    t_vjp = prof["vjp"][0] + prof["vjp_lift"][0]
    # one Runge-Kutta step against its reverse (which recomputes the stages)
    V, Vb = U0.clone(), torch.empty_like(U0)

    def wall_of(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_step = wall_of(lambda: op.rk_step(V, dt))
    t_step_vjp = wall_of(lambda: op.rk_step_vjp(U0, dt, lam, out=Vb))
    op.close()
    return {"workload": "TGV Ma0.1 Re1600, N=5, 16^3 elems, PI+Roe, BR1; d KE(t_200)/d U_0, checkpoints every 20",
            "steps": steps, "forward_s": t_fwd, "gradient_s": t_grad, "gradient_over_forward": t_grad / t_fwd,
            "vjp_over_operator_kernel_time": t_vjp / t_op, "rk_step_vjp_over_rk_step": t_step_vjp / t_step,
            "fd_check": {"eps": eps, "directions": n_dirs, "max_rel_err": max(errs), "rel_errs": errs}}


def vjp_only(torch, dg, inputs, reps=10):
    """One reverse product (dg_vjp) against one operator evaluation on the
    adjoint configuration's mesh (TGV N = 5, 16^3, symmetry-broken), without
    the rollout: the launches a kernel profile of the reverse kernels needs."""
    N, nelem, mu = 5, (16, 16, 16), 1.0 / 1600
    op = dg.DG(nelem, N, gamma=1.4, mu=mu, equations=dg.NS, vol_flux=dg.PI, surf_flux=dg.ROE, Pr=0.72)
    U0 = torch.from_numpy(inputs.tgv(N, nelem, symmetry_break=True)).to("cuda:0")
    lam = torch.from_numpy(inputs.random_directions(tuple(U0.shape), 99)).to("cuda:0")
    out = torch.empty_like(U0)
    op.time_derivative(U0)  # first launches (code object loading) outside the timed ones
    op.vjp(U0, lam, out=out)
    torch.cuda.synchronize()
    op.set_profiling(True)
    for _ in range(reps):
        op.time_derivative(U0)
        op.vjp(U0, lam, out=out)
    prof = op.profile_read()
    op.close()
    t_op = prof["stage"][0] + prof["lift"][0]
    t_vjp = prof["vjp"][0] + prof["vjp_lift"][0]
    return {"workload": "TGV Ma0.1 Re1600, N=5, 16^3 elems, PI+Roe, BR1; dg_vjp vs dg_time_derivative",
            "reps": reps, "operator_ms": t_op / reps, "vjp_ms": t_vjp / reps, "vjp_over_operator": t_vjp / t_op,
            "kernel_ms": {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]}}


def cpu_baseline(name, spec, U0, dt, max_nodes=8_000_000):
    """The oracle timed on the host cores: one LSERK4 step of the workload; for
    meshes above max_nodes the same flow on a mesh with fewer elements per
    direction (same N, same per-node work) so the sample stays near 10-30 s.
    Also one core on an eighth of that sample (PID per core, for comparison
    with the paper's per-core figures)."""
    from oracle import oracle as orc
    N, nelem, eq, vf, sf, mu, blend, _ = spec
    lo, hi = domain(name)
    cores = len(os.sched_getaffinity(0))
    sample_elems = tuple(nelem)
    U = U0
    while int(np.prod(sample_elems)) * (N + 1) ** 3 > max_nodes:
        sample_elems = tuple(max(1, n // 2) for n in sample_elems)
    if sample_elems != tuple(nelem) or U is None:
        U = initial_state(name, N, sample_elems)

    def run(elems, U, threads):
        orc.set_threads(threads)
        wd, ui, mi = WALLS.get(name, (-1, 1.0, 0.0))
        s = orc.Setup(N=N, nelem=elems, lo=lo, hi=hi, equations=eq, vol_flux=vf, surf_flux=sf, mu=mu,
                      blending=blend, Pr=0.72, Cs=MODEL_CS.get(name, 0.0), xnodes=curved_nodes(name, N, elems),
                      wall_dir=wd, wm_uinf=ui, wm_mainf=mi)
        t0 = time.perf_counter()
        orc.rk_steps(s, U, dt, 1)
        return time.perf_counter() - t0

    nodes = U.shape[0] * (N + 1) ** 3
    wall = run(sample_elems, U, cores)
    one_elems = tuple(max(1, n // 2) for n in sample_elems)
    U1 = initial_state(name, N, one_elems)
    nodes1 = U1.shape[0] * (N + 1) ** 3
    wall1 = run(one_elems, U1, 1)
    orc.set_threads(cores)
    what = "full mesh" if sample_elems == tuple(nelem) else f"same flow on {sample_elems} elements"
    return {"value": nodes * 5 / wall, "unit": "DOF-stage/s", "cores": cores, "kind": "oracle",
            "sample": f"1 LSERK4 step (5 operator evaluations), {what}, {nodes} DOF, {wall:.1f} s wall",
            "pid_us_per_core": wall * cores / (nodes * 5) * 1e6,
            "one_core": {"pid_us": wall1 / (nodes1 * 5) * 1e6,
                         "sample": f"1 LSERK4 step on {one_elems} elements, {nodes1} DOF, {wall1:.1f} s wall"}}


def device_freestream(torch, N, nelem, gamma=1.4, rho=1.0, u=0.5, p=None):
    """Constant state rho = 1, u = (0.5, 0, 0), p = 1/gamma built directly in
    device memory (the largest sweep meshes would need tens of GB of host RAM)."""
    p = 1.0 / gamma if p is None else p
    n1 = N + 1
    U = torch.empty((int(np.prod(nelem)), 5, n1, n1, n1), dtype=torch.float64, device="cuda:0")
    for v, val in enumerate((rho, rho * u, 0.0, 0.0, p / (gamma - 1.0) + 0.5 * rho * u * u)):
        U[:, v].fill_(val)
    return U


def timed_rollouts(torch, op, U, dt, steps, warmup, repeats, profile):
    """`warmup` untimed steps, then `repeats` blocks of exactly `steps` steps,
    each bracketed by device synchronisation.  Per-kernel event times are
    collected over the first block only."""
    if warmup:
        op.rk_steps(U, dt, warmup)
    walls, prof = [], None
    for r in range(repeats):
        op.set_profiling(profile and r == 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op.rk_steps(U, dt, steps)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        if profile and r == 0:
            prof = op.profile_read()
    op.set_profiling(False)
    return walls, prof


def repeat_stats(nodes, steps, walls):
    vals = [nodes * 5 * steps / w for w in walls]
    return {"n": len(vals), "mean": float(np.mean(vals)), "min": float(np.min(vals)), "max": float(np.max(vals))}


def measured_copy_bandwidth(torch, mib=4096, reps=10):
    """Achievable HBM bandwidth on this device: a plain device-to-device copy
    of a float64 buffer (read + write bytes over the event-timed copies)."""
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * 8 * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def face_flux_bytes_per_node(N, viscous, split):
    """Algorithmic bytes per node and stage launch of the normal viscous face
    flux (FP64, 4 values at each of the 6 (N+1)^2 face nodes of an element):
    the stage kernel reads the neighbours' (192/(N+1) B per node); with the
    split lifting it also writes the own part of its output in stages 1-4."""
    if not viscous:
        return 0.0
    f = 192.0 / (N + 1)
    return f * (1.0 + (0.8 if split else 0.0))


def roofline(name, nodes, steps, prof, N=None, viscous=False, split=False):
    """Roofline of the stage kernel from its event-timed launches: achieved =
    160 B per DOF and launch (the floor of a Runge-Kutta stage:
    read U and the register, write the register and U; curved meshes add the
    80 B of metric terms) over the average launch time.  The exact per-launch
    average of the kernel (stage 1 reads no register, stage 5 writes none:
    144 B; plus the viscous face fluxes it reads and, with the split lifting,
    writes) is reported beside it."""
    ms_stage, n_stage = prof["stage"]
    avg_ms = ms_stage / max(n_stage, 1)
    extra = METRIC_BYTES_PER_NODE if name in CURVED else 0.0
    launch_bytes = (160.0 + extra) * nodes
    A = launch_bytes / (avg_ms * 1e-3) / 1e9
    face = face_flux_bytes_per_node(N, viscous, split) if N is not None else 0.0
    exact_per_node = stage_bytes_per_step(1) / 5 + extra + face
    exact = exact_per_node * nodes / (avg_ms * 1e-3) / 1e9
    traffic = None
    if name in MEASURED_TRAFFIC and kernel_sha() == MEASURED_TRAFFIC["kernel_sha"]:
        traffic = MEASURED_TRAFFIC[name]["bytes_per_launch"]
    out = {"bound": "hbm", "achieved": round(A, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(A / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_unit": "bytes per launch",
           "kernel": ("k_stage_curved" if name in CURVED else "k_stage") + " (operator + LSERK4 stage)",
           "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": launch_bytes,
           "algorithmic_bytes_per_dof": 160.0 + extra,
           "exact_bytes_per_dof": round(exact_per_node, 2),
           "frac_exact": round(exact / HBM_PEAK_GBS, 4)}
    fl = KERNEL_FLOPS.get(name)
    if fl and kernel_sha() == KERNEL_FLOPS["kernel_sha"]:
        tf = fl["stage_flops_per_dof"] * nodes / (avg_ms * 1e-3) / 1e12
        out["fp64"] = {"flops_per_dof_launch": fl["stage_flops_per_dof"], "achieved": round(tf, 2),
                       "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / FP64_PEAK_TFLOPS, 4),
                       "counted": "rocprofv3 SQ_INSTS_VALU_{FMA,ADD,MUL,TRANS}_F64 x 64 lanes per DOF"}
    return out


def blended_fraction(torch, op, U0, dt, steps, every=50):
    """Fraction of elements with alpha > 0, phi(t), along an untimed rollout."""
    U = U0.clone()
    out = []
    for k in range(0, steps + 1, every):
        if k:
            op.rk_steps(U, dt, every)
        a = op.alpha(U)
        out.append({"step": k, "t": k * dt, "phi": float((a > 0).double().mean().item()),
                    "alpha_max": float(a.max().item())})
    return out


def adjoint_timing(torch, op, U, reps=20):
    """One reverse-mode product (through the blending, or on the curved mesh)
    against one operator evaluation, wall time."""
    lam = torch.ones_like(U)

    def wall(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_op = wall(lambda: op.time_derivative(U))
    t_vjp = wall(lambda: op.vjp(U, lam))
    out = {"operator_ms": t_op * 1e3, "vjp_ms": t_vjp * 1e3, "vjp_over_operator": t_vjp / t_op}
    if op.options.blending:
        out["blended_fraction"] = float((op.alpha(U) > 0).double().mean().item())
    return out


def wall_model_cost(torch, op, U_init, dt, steps, warmup, wall):
    """Rollouts of the same start with the wall model without the van Driest
    transformation and without walls (periodic), against the wall-modelled
    run: per-step wall time and stage/lifting kernel time."""
    out = {}
    wd, ui, _ = wall
    for label, args in (("spalding_only", (wd, ui, 0.0)), ("periodic", (-1,))):
        op.set_wall_model(*args)
        U = U_init.clone()
        w, prof = timed_rollouts(torch, op, U, dt, steps, warmup, 1, True)
        out[label] = {"ms_per_step": w[0] / steps * 1e3,
                      "kernel_ms_per_step": {k: round(v[0] / steps, 4) for k, v in prof.items() if v[1]}}
        del U
    op.set_wall_model(*wall)
    return out


def sweep(torch, dg, spec, steps, warmup, repeats):
    """Freestream throughput over 2^15 ... 2^21 elements (N = 7)."""
    N, _, eq, vf, sf, mu, blend, _ = spec
    rows = []
    for nelem in SWEEP_MESHES:
        op = dg.DG(nelem, N, gamma=1.4, mu=mu, equations=eq, vol_flux=vf, surf_flux=sf, Pr=0.72)
        U = device_freestream(torch, N, nelem)
        nodes = U.shape[0] * (N + 1) ** 3
        dt = op.max_dt(U, 0.5)
        walls, prof = timed_rollouts(torch, op, U, dt, steps, warmup, repeats, True)
        row = {"elements": list(nelem), "n_elems": int(np.prod(nelem)), "dof": nodes,
               "value": nodes * 5 * steps / walls[0], "repeats": repeat_stats(nodes, steps, walls),
               "stage_roofline_frac": roofline("", nodes, steps, prof)["frac"],
               "finite_after_run": op.check_finite(U)}
        rows.append(row)
        print(json.dumps({"sweep_point": row}), file=sys.stderr, flush=True)
        op.close()
        del U
        torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed blocks of --steps steps; `value` is the first, the rest give mean/min/max")
    ap.add_argument("--workload", default="tgv_n7_64", choices=sorted(WORKLOADS))
    ap.add_argument("--sweep", action="store_true",
                    help="freestream workloads: also time 2^15 ... 2^21 elements")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint (gradient) leg")
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--lifting", choices=("split", "two_pass"), default="split",
                    help="BR1 lifting scheme of the Navier-Stokes operator (split: the library default)")
    ap.add_argument("--no-lifting-compare", action="store_true",
                    help="skip the one-block run with the other lifting scheme")
    ap.add_argument("--vjp-only", action="store_true",
                    help="only time dg_vjp against dg_time_derivative on the adjoint mesh (N = 5, 16^3) and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized float64 device buffer 5 times (reference kernel for the "
                         "FETCH_SIZE/WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read_per_launch": n * 8, "bytes_written_per_launch": n * 8,
                          "launches": 5}))
        return
    if args.vjp_only:
        import torch

        from paper_2306_12891_amd import dg, inputs
        print(json.dumps(vjp_only(torch, dg, inputs)))
        return
    if args.gpus != 1:
        print(f"bench.py: this path runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU element decomposition is a design only)", file=sys.stderr)
        sys.exit(2)
    repeats = max(1, args.repeats)

    import torch

    from paper_2306_12891_amd import dg

    name = args.workload
    spec = WORKLOADS[name]
    N, nelem, eq, vf, sf, mu, blend, desc = spec
    lo, hi = domain(name)
    nodes = int(np.prod(nelem)) * (N + 1) ** 3
    U0 = None if name.startswith("freestream") else initial_state(name, N, nelem)
    cs = MODEL_CS.get(name, 0.0)
    lifting = dg.LIFT_SPLIT if args.lifting == "split" else dg.LIFT_TWO_PASS
    op = dg.DG(nelem, N, gamma=1.4, mu=mu, lo=lo, hi=hi, equations=eq, vol_flux=vf, surf_flux=sf,
               blending=blend, Pr=0.72, Cs=cs, lifting=lifting)
    # whether the split lifting runs here (the library uses it for the FP64
    # Navier-Stokes operator on the box without eddy viscosity, blending or walls)
    split = (lifting == dg.LIFT_SPLIT and eq == dg.NS and cs == 0.0 and not blend and name not in CURVED
             and name not in WALLS)
    if name in CURVED:
        op.set_geometry(torch.from_numpy(curved_nodes(name, N, nelem)).to("cuda:0"))
    if name in WALLS:
        op.set_wall_model(*WALLS[name])
    U_init = device_freestream(torch, N, nelem) if U0 is None else torch.from_numpy(U0).to("cuda:0")
    U = U_init.clone()
    dt = op.max_dt(U, 0.5)
    walls, prof = timed_rollouts(torch, op, U, dt, args.steps, args.warmup, repeats, not args.no_profile)
    wall = walls[0]
    finite = op.check_finite(U)
    value = nodes * 5 * args.steps / wall

    roof = None
    extra = {"repeats": repeat_stats(nodes, args.steps, walls)}
    if prof:
        roof = roofline(name, nodes, args.steps, prof, N, eq == dg.NS, split)
        copy_gbs = measured_copy_bandwidth(torch)
        roof["measured_copy_GBs"] = round(copy_gbs, 1)
        roof["frac_of_measured_copy"] = round(roof["achieved"] / copy_gbs, 4)
        extra["kernel_ms_per_step"] = {k: round(v[0] / args.steps, 4) for k, v in prof.items() if v[1]}
    path_bytes = 160.0 * nodes * 5 * args.steps
    extra["path_roofline_frac_160B"] = round(path_bytes / wall / 1e9 / HBM_PEAK_GBS, 4)
    extra["pid_gpu_us"] = 1e6 / value
    extra["finite_after_run"] = finite
    # the same workload with the other BR1 lifting scheme: one block, same
    # start state and warm-up; its final state against this run's
    if (eq == dg.NS and cs == 0.0 and not blend and name not in CURVED and name not in WALLS
            and not args.no_lifting_compare):
        other = dg.LIFT_TWO_PASS if lifting == dg.LIFT_SPLIT else dg.LIFT_SPLIT
        op.set_options(lifting=other)
        Uo = U_init.clone()
        walls_o, prof_o = timed_rollouts(torch, op, Uo, dt, args.steps, args.warmup, 1, not args.no_profile)
        op.set_options(lifting=lifting)
        Uc = U_init.clone()
        op.rk_steps(Uc, dt, args.warmup + args.steps)
        scale = torch.maximum(Uc.abs().amax(dim=(0, 2, 3, 4)), Uc[:, 0].abs().amax())
        err = ((Uo - Uc).abs().amax(dim=(0, 2, 3, 4)) / scale).tolist()
        extra["other_lifting"] = {
            "lifting": "two_pass" if other == dg.LIFT_TWO_PASS else "split",
            "value": nodes * 5 * args.steps / walls_o[0], "ms_per_step": walls_o[0] / args.steps * 1e3,
            "err_vs_this_run_linf_rel": err, "after_steps": args.warmup + args.steps}
        if prof_o:
            extra["other_lifting"]["kernel_ms_per_step"] = {k: round(v[0] / args.steps, 4)
                                                            for k, v in prof_o.items() if v[1]}
            extra["other_lifting"]["stage_avg_launch_ms"] = round(prof_o["stage"][0] / max(prof_o["stage"][1], 1), 4)
        del Uo, Uc
    if blend:
        extra["blended_fraction"] = blended_fraction(torch, op, U_init, dt, args.warmup + args.steps * repeats)
        if not args.no_adjoint:
            extra["blended_adjoint"] = adjoint_timing(torch, op, U)

    # Mixed-precision operator on the same workload: same initial state, same
    # warm-up and timed steps; error of the final state against the FP64 run.
    if not args.no_mixed and vf in (1, 3) and not blend and name not in CURVED and name not in WALLS:
        opm = dg.DG(nelem, N, gamma=1.4, mu=mu, lo=lo, hi=hi, equations=eq, vol_flux=vf, surf_flux=sf,
                    Pr=0.72, precision=dg.MIXED, Cs=cs)
        # one operator evaluation at the initial state: error of the mixed U_t
        # per variable against the FP64 operator (which matches the oracle to
        # 1e-12), relative to max |U_t,v|
        ut64 = op.time_derivative(U_init)
        utm = opm.time_derivative(U_init)
        dut = (utm - ut64).abs()
        sc = ut64.abs().amax(dim=(0, 2, 3, 4))
        ut_linf = (dut.amax(dim=(0, 2, 3, 4)) / sc).tolist()
        ut_l2 = (dut.pow(2).mean(dim=(0, 2, 3, 4)).sqrt() / ut64.pow(2).mean(dim=(0, 2, 3, 4)).sqrt()).tolist()
        del ut64, utm, dut
        Um = U_init.clone()
        walls_m, profm = timed_rollouts(torch, opm, Um, dt, args.steps, args.warmup, repeats,
                                        not args.no_profile)
        wall_m = walls_m[0]
        diff = (Um - U).abs()
        scale = torch.maximum(U.abs().amax(dim=(0, 2, 3, 4)), U[:, 0].abs().amax())
        linf = (diff.amax(dim=(0, 2, 3, 4)) / scale).tolist()
        l2 = (diff.pow(2).mean(dim=(0, 2, 3, 4)).sqrt() / scale).tolist()
        extra["mixed"] = {"value": nodes * 5 * args.steps / wall_m, "unit": "DOF-stage/s",
                          "repeats": repeat_stats(nodes, args.steps, walls_m),
                          "ms_per_step": wall_m / args.steps * 1e3, "speedup_vs_fp64": wall / wall_m,
                          "err_vs_fp64_linf_rel": linf, "err_vs_fp64_l2_rel": l2,
                          "err_bound_stated": 1e-5, "within_bound": max(linf) <= 1e-5,
                          "after_steps": args.warmup + args.steps * repeats,
                          "ut_err_linf_rel_max_ut": ut_linf, "ut_err_l2_rel": ut_l2,
                          "ut_err_note": "one evaluation at the initial state against the FP64 operator; rho and E "
                                         "rates at Ma 0.1 are small differences of O(p0), O(h0) flux terms"}
        if profm:
            extra["mixed"]["kernel_ms_per_step"] = {k: round(v[0] / args.steps, 4) for k, v in profm.items() if v[1]}
            extra["mixed"]["stage_roofline_frac"] = roofline("", nodes, args.steps, profm)["frac"]
        opm.close()
        del Um

    if name in WALLS:
        if prof:
            extra["wall_model_cost"] = wall_model_cost(torch, op, U_init, dt, args.steps, args.warmup, WALLS[name])
    elif not args.no_adjoint and name in CURVED:
        extra["curved_adjoint"] = adjoint_timing(torch, op, U)
    elif not args.no_adjoint:
        from paper_2306_12891_amd import inputs
        extra["adjoint"] = adjoint_leg(torch, dg, inputs)

    if args.sweep and name.startswith("freestream"):
        op.close()
        op = None
        del U, U_init
        torch.cuda.empty_cache()
        extra["sweep"] = sweep(torch, dg, spec, args.steps, args.warmup, repeats)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(name, spec, U0, dt)

    line = {
        "metric": METRIC, "value": value, "unit": "DOF-stage/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "N": N, "elements": list(nelem), "dof": nodes, "dt": dt,
                   "precision": "fp64", "br1_lifting": ("split" if split else "two_pass") if eq == dg.NS else None},
        "roofline": roof, "cpu_baseline": cpu, **extra,
    }
    print(json.dumps(line))
    if op is not None:
        op.close()


if __name__ == "__main__":
    main()
