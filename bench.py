"""Throughput of the COLA PM step on one MI355X.

Workload (default): 1024^3 particles, 2048^3 PM mesh (2x the particle grid),
1200 Mpc/h box, flat LCDM Omega_m = 0.27, BBKS P(k) with sigma_8 = 0.8,
Gaussian white-noise initial conditions (GPU Philox, seed 5) displaced by
2LPT, 10 COLA steps uniform in a from 0.02 to 1.  A "step" is one
cola_step: tile sort, deterministic CIC deposit, r2c FFT, Green's function
x ik and the inverse FFTs of the three force components, CIC readout fused
with the kick/drift.  ``--config production`` selects 256^3 / 768^3 / 600
Mpc/h instead.

Timed region: K steps of the 10-step schedule, cycled: every pass of up to
10 steps starts from fresh initial conditions (cola_init_2lpt, outside the
timer), inputs resident in HBM, each pass bracketed by
torch.cuda.synchronize(); the timed passes are summed.  W untimed warm-up
steps come first, in the same cycle.

Then, each in its own pass:
* fwd_adjoint -- the gradient of the final P(k) (40 log bins, seeded
  cotangents) with respect to the white noise.  Large runs use the lean
  driver (autograd.pk_noise_gradient: one position buffer, step starts
  recomputed from the initial conditions); smaller ones reverse K steps from
  stored starts, and also store the forces instead of recomputing them
  (fwd_adjoint_kept) where the slots fit in HBM.
* roofline -- the library's per-stage HIP event timers (on the library's
  stream) over the 10-step schedule give each stage's average launch time;
  the dominant kernel's algorithmic bytes over that time, against 8 TB/s.
  ``traffic`` comes from the committed rocprofv3 counter summary of this
  workload while its kernel sources are unchanged.
* production -- with the large workload, the same measurements at
  256^3 / 768^3 (velocity, snapshot, velocity spectra, friends-of-friends
  legs included).
* batched -- the 96-mock ensemble batched and one by one.
* cpu_baseline -- one FP64 oracle step on a sub-volume of the workload at
  its resolution (host cores).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    """Progress of the legs on stderr (the JSON line is the only stdout)."""
    print("[bench]", *a, file=sys.stderr, flush=True)
# host memory the full FP64 oracle run of a workload needs (particles, two
# meshes and temporaries in FP64), for the P(k) parity note
ORACLE_HOST_BYTES_PER_NODE = 40.0


def stage_bytes(np_side: int, nm: int) -> dict:
    """Algorithmic HBM bytes per launch of each stage (what the method must move)."""
    n_p = np_side ** 3
    M = nm ** 3
    R = 4 * M                               # real float32 mesh
    C = 8 * nm * nm * (nm // 2 + 1)         # complex half mesh
    return {
        "sort": 32 * n_p,                   # read d (12), write+read key/rank (16), write perm (4)
        "deposit": 16 * n_p + R,            # read perm + d, write delta
        "fft_z": R + C,                     # real in, half spectrum out
        "fft_y": 2 * C,
        "fft_x_green": 3 * C,               # 1 read, 2 writes (IDFT_x of i k_x phi and of phi)
        "ifft_y": 2 * C,                    # g_x: read + write
        "ifft_y_grad": 3 * C,               # IDFT_x[phi]: 1 read, 2 writes (g_y, g_z)
        "ifft_z": 3 * (C + R),              # three meshes, half spectrum in, real out
        "kick_drift": 72 * n_p + 3 * 4 * min(M, 8 * n_p),  # state r/w + CIC gathers
    }


STAGE_SOURCES = {
    "sort": ["k_sort.hip"], "deposit": ["k_deposit.hip"], "fft_z": ["k_fft.hip"],
    "fft_y": ["k_fft.hip"], "fft_x_green": ["k_fft.hip"], "ifft_y": ["k_fft.hip"],
    "ifft_z": ["k_fft.hip"], "ifft_y_grad": ["k_fft.hip"], "kick_drift": ["k_particles.hip"],
}


def traffic_file(np_side, nm):
    """Committed counter summary (rocprofv3 FETCH_SIZE / WRITE_SIZE) of a workload."""
    return os.path.join(ROOT, "profiles", f"hbm_traffic_{np_side}p_{nm}m.txt")


def measured_traffic(stage, np_side, nm):
    """HBM bytes per launch of a stage from the committed counter summary, or
    None when there is none for this workload or the kernel source changed."""
    import hashlib
    path = traffic_file(np_side, nm)
    if not os.path.exists(path):
        return None
    sha, traffic = {}, {}
    for line in open(path):
        f = line.split()
        if len(f) == 3 and f[0] == "sha256":
            sha[f[1]] = f[2]
        elif len(f) >= 3 and f[0] == "traffic":
            traffic[f[1]] = int(f[2])
    if stage not in traffic:
        return None
    csrc = os.path.join(ROOT, "paper_1507_05329_amd", "csrc")
    for name in STAGE_SOURCES.get(stage, []) + ["cola_device.h"]:
        h = hashlib.sha256(open(os.path.join(csrc, name), "rb").read()).hexdigest()
        if sha.get(name) != h:
            return None
    return traffic[stage]


def host_info():
    """CPU model, host RAM and the cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal:"):
                ram = int(line.split()[1]) * 1024
                break
    except OSError:
        pass
    return {"cpu_model": model, "ram_GB": None if ram is None else round(ram / 1e9, 1),
            "cores": len(os.sched_getaffinity(0))}


def cycled_steps(sim, cfg, table, e, nsteps):
    """Runs nsteps steps of the cfg.nstep-step schedule, cycled: each pass of
    up to cfg.nstep steps starts from fresh initial conditions (untimed).
    Returns the summed wall time of the passes (device synchronised)."""
    import torch
    total = 0.0
    done = 0
    while done < nsteps:
        sim.init_2lpt(cfg.seed, *table)
        n = min(cfg.nstep, nsteps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n):
            sim.step(e[i], e[i + 1])
        torch.cuda.synchronize()
        total += time.perf_counter() - t0
        done += n
    return total


def stage_pass(cfg, table, e, dev, with_outputs):
    """Per-stage averages over the whole schedule from the library's HIP event
    timers; optionally the velocity / snapshot / spectra / FoF legs at the end."""
    from paper_1507_05329_amd import _lib
    from paper_1507_05329_amd.sim import ColaSim
    simt = ColaSim(cfg.np_side, cfg.nmesh, cfg.box, omega_m=cfg.omega_m, n_lpt=cfg.n_lpt,
                   a_init=cfg.a_init, device=dev, flags=_lib.COLA_F_STAGE_TIMERS)
    try:
        simt.init_2lpt(cfg.seed, *table)
        simt.synchronize()
        simt.stage_times()
        for i in range(cfg.nstep):
            simt.step(e[i], e[i + 1])
        st = simt.stage_times()
        extra = {}
        if with_outputs:
            extra["velocity"] = velocity_leg(simt, cfg)
            extra["fof"] = fof_leg(simt)
    finally:
        simt.close()
    sb = stage_bytes(cfg.np_side, cfg.nmesh)
    stages = {}
    for name, (ms, cnt) in st.items():
        if cnt == 0 or name not in sb:
            continue
        avg = ms / cnt
        stages[name] = {"ms": round(avg, 4), "launches": cnt,
                        "GB/s": round(sb[name] / (avg * 1e-3) / 1e9, 1)}
    return stages, extra


def roofline_of(stages, cfg, ms_step):
    sb = stage_bytes(cfg.np_side, cfg.nmesh)
    dom = max(stages, key=lambda n: stages[n]["ms"])
    dom_gbs = sb[dom] / (stages[dom]["ms"] * 1e-3) / 1e9
    step_bytes = sum(sb.values())
    return {"bound": "hbm", "kernel": dom, "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom, cfg.np_side, cfg.nmesh),
            "bytes_alg": sb[dom], "ms_per_launch": stages[dom]["ms"],
            "step_bytes_alg": step_bytes,
            "step_frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def velocity_leg(sim, cfg, reps=3):
    """cola_velocity at the final state (a_v != a_x, so the call runs the force
    pipeline, then the velocity kernel with a redshift-space output): whole-call
    time and the kernel's own time from the stage timers (HIP events on the
    library's stream) against its algorithmic bytes."""
    import numpy as np
    import torch
    vel, sdisp = sim.particles(), sim.particles()
    sim.velocity(vel, rsd_axis=2, sdisp=sdisp)
    torch.cuda.synchronize()
    sim.stage_times()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.velocity(vel, rsd_axis=2, sdisp=sdisp)
    torch.cuda.synchronize()
    ms_call = (time.perf_counter() - t0) / reps * 1e3
    ms, cnt = sim.stage_times()["velocity"]
    ms_k = ms / max(cnt, 1)
    n_p, M = cfg.np_side ** 3, cfg.nmesh ** 3
    nbytes = 72 * n_p + 12 * min(M, 8 * n_p)   # state reads 48, outputs 24, CIC gathers
    st = sim.get_state(which=())
    a1 = st["a_x"] + 0.098
    sim.snapshot(a1, st["a_x"] + 0.049)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.snapshot(a1, st["a_x"] + 0.049)
    torch.cuda.synchronize()
    ms_snap = (time.perf_counter() - t0) / reps * 1e3
    edges = np.linspace(2 * np.pi / cfg.box, np.pi * cfg.nmesh / cfg.box, 41)
    sim.pk_velocity(edges, axis=2)
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.pk_velocity(edges, axis=2)
    ms_pkv = (time.perf_counter() - t0) / reps * 1e3
    return {"ms_call": round(ms_call, 3), "ms_kernel": round(ms_k, 4), "bytes_alg": nbytes,
            "GB/s": round(nbytes / (ms_k * 1e-3) / 1e9, 1),
            "ms_snapshot_call": round(ms_snap, 3), "ms_pk_velocity_call": round(ms_pkv, 3),
            "note": "velocity at the position time plus the redshift-space displacement (axis 2); "
                    "each call includes the force pipeline at the current positions; pk_velocity "
                    "adds the weighted deposit, 2 FFTs and 40-bin spectra (synchronous)"}


def fof_leg(sim, reps=3):
    """cola_fof (b = 0.2 of the mean separation) at the final positions: time per
    call (the call synchronises) and the groups of at least 32 particles."""
    import torch
    lab = sim.fof(0.2)
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.fof(0.2, out=lab)
    ms = (time.perf_counter() - t0) / reps * 1e3
    sizes = torch.bincount(lab.long())
    big = sizes >= 32
    vel = sim.velocity()
    sim.fof_halos(lab, vel, min_members=32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        cat = sim.fof_halos(lab, vel, min_members=32)
    ms_cat = (time.perf_counter() - t0) / reps * 1e3
    return {"ms_call": round(ms, 3), "ms_catalogue_call": round(ms_cat, 3), "halos": int(cat["root"].numel()),
            "b_frac": 0.2, "groups_ge_32": int(big.sum()),
            "frac_in_groups_ge_32": round(float(sizes[big].sum()) / lab.numel(), 4),
            "largest": int(sizes.max())}


def batch_leg(steps, table, dev):
    """The 96-mock uneven ensemble (32 x 48^3/96^3, 32 x 64^3/128^3,
    32 x 96^3/192^3 particles/mesh, boxes 150/200/300 Mpc/h, distinct seeds):
    the 10-step run batched (one graph per step) against the same mocks
    stepped one by one with plain contexts."""
    import torch
    from paper_1507_05329_amd.inputs import batch_configs, step_edges
    from paper_1507_05329_amd.sim import ColaBatch, ColaSim
    cfgs = batch_configs()
    e = step_edges()
    n_part = sum(c.n_particles for c in cfgs)
    b = ColaBatch([dict(np=c.np_side, nmesh=c.nmesh, box=c.box) for c in cfgs], device=dev)
    tuned = {}
    for m, c in zip(b.mocks, cfgs):
        if c.nmesh not in tuned:
            tuned[c.nmesh] = m.autotune(reps=3)[0]
    for m, c in zip(b.mocks, cfgs):
        m.init_2lpt(c.seed, *table)
    b.step(e[0], e[1])                      # warm-up; captures the graph
    for m, c in zip(b.mocks, cfgs):
        m.init_2lpt(c.seed, *table)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        b.step(e[i], e[i + 1])
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    b.close()
    del b
    sims = {}
    t_seq = 0.0
    for c in cfgs:
        key = (c.np_side, c.nmesh, c.box)
        if key not in sims:
            sims[key] = ColaSim(c.np_side, c.nmesh, c.box, device=dev)
            sims[key].init_2lpt(c.seed, *table)
            sims[key].step(e[0], e[1])      # warm-up of this size
        s = sims[key]
        s.init_2lpt(c.seed, *table)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            s.step(e[i], e[i + 1])
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
    for s in sims.values():
        s.close()
    return {"workload": "96 mocks: 32 x 48^3/96^3 (150 Mpc/h), 32 x 64^3/128^3 (200), "
                        "32 x 96^3/192^3 (300), distinct seeds",
            "mocks": len(cfgs), "particles": n_part, "steps": steps,
            "value": n_part * steps / t_batch, "unit": "particle-updates/s",
            "ms_per_step": t_batch / steps * 1e3,
            "sequential_value": n_part * steps / t_seq,
            "sequential_ms_per_step": t_seq / steps * 1e3,
            "speedup": t_seq / t_batch,
            "fft_block_order": {str(k): v for k, v in tuned.items()}}


def adjoint_leg(sim, cfg, table, e, steps):
    """Average adjoint step (ms): reverse the first `steps` steps from their
    stored starts (displacements only)."""
    import torch
    sim.init_2lpt(cfg.seed, *table)
    starts = []
    for i in range(steps):
        st = sim.get_state(("disp",))
        starts.append((st["disp"], st["a_v"]))
        sim.step(e[i], e[i + 1])
    dbar = torch.randn_like(starts[0][0])
    vbar = torch.zeros_like(dbar)
    p1b, p2b = torch.zeros_like(dbar), torch.zeros_like(dbar)
    sim.step_adjoint(e[steps - 1], e[steps], starts[-1][1], starts[-1][0], dbar, vbar, p1b, p2b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in reversed(range(steps)):
        sim.step_adjoint(e[i], e[i + 1], starts[i][1], starts[i][0], dbar, vbar, p1b, p2b)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def kept_leg(sim, cfg, table, e, steps):
    """Store instead of recompute: the forward steps keep their force meshes
    (cola_step_keep, one slot per step) and the adjoint reads them
    (cola_step_adjoint_kept).  Returns (ms per forward step, ms per adjoint
    step, GB of slots), or None when the slots do not fit in free HBM."""
    import torch
    slots = [sim.force_slot()]
    per = slots[0].numel() * 4
    free, _ = torch.cuda.mem_get_info()
    if (steps - 1) * per > 0.8 * free:
        return None
    slots += [sim.force_slot() for _ in range(steps - 1)]
    sim.init_2lpt(cfg.seed, *table)
    starts = []
    torch.cuda.synchronize()
    t_fwd = 0.0
    for i in range(steps):
        st = sim.get_state(("disp",))
        starts.append((st["disp"], st["a_v"]))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step_keep(e[i], e[i + 1], slots[i])
        torch.cuda.synchronize()
        t_fwd += time.perf_counter() - t0
    dbar = torch.randn_like(starts[0][0])
    vbar = torch.zeros_like(dbar)
    p1b, p2b = torch.zeros_like(dbar), torch.zeros_like(dbar)
    sim.step_adjoint(e[steps - 1], e[steps], starts[-1][1], starts[-1][0], dbar, vbar, p1b, p2b,
                     slot=slots[-1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in reversed(range(steps)):
        sim.step_adjoint(e[i], e[i + 1], starts[i][1], starts[i][0], dbar, vbar, p1b, p2b, slot=slots[i])
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    gb = steps * per / 1e9
    del slots
    torch.cuda.empty_cache()
    return t_fwd / steps * 1e3, t_adj / steps * 1e3, gb


def lean_gradient_leg(sim, cfg, table, e, ms_step):
    """The gradient of sum_b c_b P_b (40 log bins from 2 pi / L to the mesh
    Nyquist, c_b ~ N(0, 1) seed 5) with respect to the white noise through the
    lean driver: forward run, then for every step (last first) its start
    recomputed from the initial conditions and its adjoint."""
    import numpy as np
    import torch
    from paper_1507_05329_amd.autograd import pk_noise_gradient
    from paper_1507_05329_amd.inputs import seeded_normal
    kf, kny = 2 * np.pi / cfg.box, np.pi * cfg.nmesh / cfg.box
    kedges = np.exp(np.linspace(np.log(kf), np.log(kny), 41))
    cbar = seeded_normal(5, (40,)).astype(np.float64)
    noise = sim.noise(cfg.seed)
    times = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, _ = pk_noise_gradient(sim, noise, table[0], table[1], e, kedges, cbar, times=times)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    finite = bool(torch.isfinite(g).all().item())
    del g, noise
    torch.cuda.empty_cache()
    n = cfg.nstep
    ms_adj = times["adjoint"] / n * 1e3
    backward = total - times["forward"]
    return {"value": cfg.n_particles / ((ms_step + backward / n * 1e3) * 1e-3), "unit": "particle-updates/s",
            "ms_adjoint_step": round(ms_adj, 3), "adjoint_over_forward": round(ms_adj / ms_step, 3),
            "ms_backward_per_step_amortised": round(backward / n * 1e3, 3),
            "s_gradient_total": round(total, 3), "s_forward": round(times["forward"], 3),
            "s_recompute": round(times["recompute"], 3), "recomputed_steps": times["recomputed_steps"],
            "gradient_finite": finite,
            "note": "lean driver: step starts recomputed from the initial conditions, no checkpoints; "
                    "value = particles / (forward step + amortised backward per step)"}


def workload_block(cfg, steps, warmup, dev, with_adjoint, with_outputs, lean):
    """Forward throughput, adjoint and per-stage timing of one workload."""
    import torch
    from paper_1507_05329_amd.inputs import bbks_table, step_edges
    from paper_1507_05329_amd.sim import ColaSim
    table = bbks_table(cfg.omega_m, cfg.h, cfg.n_s, cfg.sigma8)
    e = step_edges(cfg.a_init, cfg.a_final, cfg.nstep)
    sim = ColaSim(cfg.np_side, cfg.nmesh, cfg.box, omega_m=cfg.omega_m, n_lpt=cfg.n_lpt,
                  a_init=cfg.a_init, device=dev)
    out = {}
    try:
        best, ms = sim.autotune(reps=3)
        out["fft_schedule"] = {"n": cfg.nmesh, "block_order": best,
                               "ms_by_pass_and_order": {f"{k}/{o}": round(v, 4) for (k, o), v in ms.items()}}
        log(f"{cfg.np_side}^3/{cfg.nmesh}^3: autotune {best} {ms}")
        if warmup:
            cycled_steps(sim, cfg, table, e, warmup)
        log(f"{cfg.np_side}^3/{cfg.nmesh}^3: {warmup} warm-up steps done")
        dt = cycled_steps(sim, cfg, table, e, steps)
        ms_step = dt / steps * 1e3
        out.update(value=cfg.n_particles * steps / dt, ms_per_step=ms_step)
        log(f"{cfg.np_side}^3/{cfg.nmesh}^3: {steps} timed steps, {ms_step:.2f} ms/step")
        if with_adjoint:
            if lean:
                out["fwd_adjoint"] = lean_gradient_leg(sim, cfg, table, e, ms_step)
            else:
                n = cfg.nstep
                ms_adj = adjoint_leg(sim, cfg, table, e, n)
                out["fwd_adjoint"] = {"value": cfg.n_particles / ((ms_step + ms_adj) * 1e-3),
                                      "unit": "particle-updates/s", "ms_adjoint_step": ms_adj,
                                      "adjoint_over_forward": ms_adj / ms_step,
                                      "note": f"the {n} adjoint steps from stored step starts"}
                kept = kept_leg(sim, cfg, table, e, n)
                out["fwd_adjoint_kept"] = None if kept is None else {
                    "value": cfg.n_particles / ((kept[0] + kept[1]) * 1e-3), "unit": "particle-updates/s",
                    "ms_forward_step": kept[0], "ms_adjoint_step": kept[1], "slots_GB": kept[2],
                    "note": "forward steps keep their force meshes (one slot per step); the adjoint reads them"}
            log(f"{cfg.np_side}^3/{cfg.nmesh}^3: adjoint legs done")
    finally:
        sim.close()
        del sim
        torch.cuda.empty_cache()
    stages, extra = stage_pass(cfg, table, e, dev, with_outputs)
    torch.cuda.empty_cache()
    log(f"{cfg.np_side}^3/{cfg.nmesh}^3: stage timers done")
    out["stages"] = stages
    out["roofline"] = roofline_of(stages, cfg, out["ms_per_step"])
    out.update(extra)
    return out


def cpu_baseline(cfg):
    """One FP64 oracle COLA step (NumPy/SciPy) on the host: the workload
    itself when it has at most 256^3 particles, else a sub-volume at the
    same particle and mesh spacing (256^3 particles, box scaled down)."""
    from oracle import cola
    from paper_1507_05329_amd.inputs import bbks_table, step_edges, white_noise
    table = bbks_table(cfg.omega_m, cfg.h, cfg.n_s, cfg.sigma8)
    n, m, box = cfg.np_side, cfg.nmesh, cfg.box
    if n > 256:
        f = n // 256
        n, m, box = n // f, m // f, box / f
    w = white_noise(cfg.seed, n)
    st = cola.init_state(w, box, m, *table)
    e = step_edges(cfg.a_init, cfg.a_final, cfg.nstep)
    t0 = time.perf_counter()
    cola.step(st, e[1])
    dt = time.perf_counter() - t0
    info = host_info()
    sub = "" if (n, m) == (cfg.np_side, cfg.nmesh) else \
        f" (a 1/{(cfg.np_side // n) ** 3} sub-volume of the {cfg.np_side}^3/{cfg.nmesh}^3 workload at its " \
        f"particle and mesh spacing)"
    return {"value": n ** 3 / dt, "unit": "particle-updates/s", "cores": info["cores"],
            "kind": "oracle", "cpu_model": info["cpu_model"], "ram_GB": info["ram_GB"],
            "config": {"np": n, "nmesh": m, "box": box},
            "sample": f"one FP64 oracle COLA step (a {e[0]:.3f}->{e[1]:.3f}) of {n}^3 particles on a "
                      f"{m}^3 mesh, box {box:g} Mpc/h{sub}: {dt:.1f} s, scipy.fft workers={info['cores']}"}


def pk_parity_note(cfg):
    need = ORACLE_HOST_BYTES_PER_NODE * cfg.nmesh ** 3
    ram = host_info()["ram_GB"]
    if ram is not None and need / 1e9 < 0.8 * ram:
        return None
    return (f"final P(k) parity with the FP64 oracle unverified at this size: the full oracle run needs "
            f"about {need / 1e9:.0f} GB of host memory, this host has {ram} GB; the same kernels are "
            f"parity-tested at every other length and the sampled-node / growth checks run here")


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="large", choices=["small", "production", "diff", "large"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-ensemble leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint legs")
    ap.add_argument("--no-velocity", action="store_true", help="skip the velocity / redshift-space / FoF legs")
    ap.add_argument("--no-production", action="store_true",
                    help="with the large workload, skip the secondary 256^3/768^3 block")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (for HBM counter "
                         "calibration under rocprofv3) and exit")
    return ap.parse_args(argv)


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py: this benchmark measures one GPU; --gpus {args.gpus} is not supported "
              "(the library runs one context per GPU and has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: --steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration_mib:
        import torch
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_calibration_mib, "launches": 3}))
        return

    import torch
    from paper_1507_05329_amd import _lib
    from paper_1507_05329_amd.inputs import CONFIGS, bbks_table

    _lib.load()
    cfg = CONFIGS[args.config]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    large = cfg.n_particles > 256 ** 3

    main_block = workload_block(cfg, args.steps, args.warmup, dev, not args.no_adjoint,
                                with_outputs=not large and not args.no_velocity, lean=large)
    production = None
    if large and not args.no_production:
        pcfg = CONFIGS["production"]
        production = workload_block(pcfg, min(args.steps, pcfg.nstep), min(args.warmup, 3), dev,
                                    not args.no_adjoint, with_outputs=not args.no_velocity, lean=False)
        production["config"] = {"workload": pcfg.name, "np": pcfg.np_side, "nmesh": pcfg.nmesh,
                                "box": pcfg.box}
        production["steps"] = min(args.steps, pcfg.nstep)

    batched = None
    if not args.no_batch:
        batched = batch_leg(10, bbks_table(), dev)
        log("batched ensemble done")

    cpu = None if args.no_cpu_baseline else cpu_baseline(cfg)
    log("cpu baseline done")

    out = {
        "metric": "particle-updates/s per COLA PM step (fwd; fwd+adjoint in fwd_adjoint) + % HBM roofline",
        "value": main_block["value"],
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_block["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (BBKS Gaussian random field, GPU Philox seed %d)" % cfg.seed,
        "config": {"workload": cfg.name, "np": cfg.np_side, "nmesh": cfg.nmesh, "box": cfg.box,
                   "nstep": cfg.nstep, "a": [cfg.a_init, cfg.a_final],
                   "schedule": "the 10-step schedule cycled; fresh initial conditions (untimed) "
                               "before every pass of 10 steps"},
        "fwd_adjoint": main_block.get("fwd_adjoint"),
        "fwd_adjoint_kept": main_block.get("fwd_adjoint_kept"),
        "fft_schedule": main_block.get("fft_schedule"),
        "stages": main_block["stages"],
        "roofline": main_block["roofline"],
        "pk_parity": pk_parity_note(cfg),
        "velocity": main_block.get("velocity"),
        "fof": main_block.get("fof"),
        "production": production,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
