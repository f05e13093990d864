#!/usr/bin/env python3
"""Throughput benchmark of the two-component D3Q19 Shan-Chen step on one MI355X.

One step = one call of lb_step(1): densities and pseudopotentials, force,
velocity-shifted BGK collision, streaming, for both components of every
node.  Default workload: the 256^3 periodic spinodal lattice in float64
(tau = 0.8, G = 3.5, rho_A, rho_B = 1 +- 0.02 uniform noise).  GLUPS counts
nodes, solid or not, per second (Eq. glups of the paper).

Prints one JSON line.  Inputs are synthetic and already resident in HBM when
the timed region starts.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "GLUPS & % HBM roofline, 2-comp D3Q19 256^3; adjoint/forward time ratio"
BYTES_PER_VALUE = {"f64": 8, "f32": 4, "f16s": 2}
KERNEL_SOURCES = ["paper_2112_08264_amd/csrc/lb_device.h", "paper_2112_08264_amd/csrc/lb_kernels.h",
                  "paper_2112_08264_amd/csrc/lb_fused.h", "paper_2112_08264_amd/csrc/lb_adjoint.h",
                  "paper_2112_08264_amd/csrc/lb_particles.h", "paper_2112_08264_amd/csrc/lb_single.h",
                  "paper_2112_08264_amd/csrc/lb_api.hip"]


def algorithmic_bytes_per_lup(storage: str) -> int:
    """Both components' 19 populations read once and written once."""
    return 2 * 19 * 2 * BYTES_PER_VALUE[storage]


def source_digest() -> str:
    """Hash of the kernel sources' code, comments and blank space left out,
    so that counters taken on a kernel stay attached to it while only its
    comments change."""
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def time_form(P, torch, w, storage: str, steps: int, warmup: int, fields, kernel="auto", timing_slots=True,
              solid=None, repeats=0, repeat_steps=300):
    """Run one storage form; return a dict of timings.  The starting totals
    are read before the warmup: the state is then still in the structure-
    of-arrays order of lb_set_fields, and the reorder into the step's own order falls in
    the warmup, not in the timed steps.  ``repeats`` more blocks of
    ``repeat_steps`` steps follow the timed region, each timed on its own."""
    a, b = fields
    lat = P.Lattice(w.shape, tau=w.tau, G=w.G, storage=storage, device=0, kernel=kernel)
    try:
        lat.set_fields(a, b, None, solid)
        tot0, _ = lat.totals()
        lat.step(warmup)
        torch.cuda.synchronize()
        P.lb_timing(lat.ctx, timing_slots)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        e0.record()
        lat.step(steps)
        e1.record()
        torch.cuda.synchronize()
        w1 = time.perf_counter()
        ev_ms = e0.elapsed_time(e1)
        kernels = {}
        for s in range(P.lb_timing_slots()):
            ms, cnt = P.lb_timing_read(lat.ctx, s)
            if cnt:
                kernels[P.lb_timing_name(s)] = {"avg_ms": ms / cnt, "launches": cnt}
        P.lb_timing(lat.ctx, False)
        repeat_ms = []
        for _ in range(repeats):
            e0.record()
            lat.step(repeat_steps)
            e1.record()
            torch.cuda.synchronize()
            repeat_ms.append(e0.elapsed_time(e1) / repeat_steps)
        tot1, nonfinite = lat.totals()
    finally:
        lat.close()
    mass_drift = max(abs(tot1[k] - tot0[k]) / abs(tot0[k]) for k in range(2))
    return {"event_ms": ev_ms, "wall_ms": (w1 - w0) * 1e3, "kernels": kernels, "nonfinite": nonfinite,
            "mass_drift": mass_drift, "repeat_ms_per_step": repeat_ms}


def _moments(torch, lat, n):
    ra = torch.empty(n, dtype=torch.float64, device="cuda")
    rb = torch.empty_like(ra)
    u = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    lat.moments(ra, rb, u)
    return ra, rb, u


def _error_row(torch, got, ref, **key):
    ra, rb, u = got
    r_a, r_b, r_u = ref
    drho = torch.maximum((ra - r_a).abs(), (rb - r_b).abs())
    return dict(key, max_drho=float(drho.max()),
                rms_drho=float(torch.sqrt(0.5 * (((ra - r_a) ** 2).mean() + ((rb - r_b) ** 2).mean()))),
                max_du=float((u - r_u).abs().max()), max_abs_u_ref=float(r_u.abs().max()))


def accuracy_run(P, torch, w, fields, checkpoints=(1, 10, 100, 1000), restart=(1, 10)):
    """Error of the float32 and float16-shifted forms against the float64 path
    (bitwise equal to the float64 oracle), measured three ways:

    * trajectory: the same initial state run by each form, compared at several
      step counts;
    * sensitivity: the float64 path itself, started from rho_A nudged by one
      ulp at every node, compared with the unperturbed float64 run.  A quench
      at G = 3.5 amplifies any difference exponentially, so once this floor
      reaches a form's trajectory error, that error measures the flow's
      sensitivity, not the storage;
    * restart: the float64 state after the last checkpoint loaded into each
      form (one rounding to its storage) and advanced a few steps, compared
      with float64 advanced the same steps -- the storage error per step in
      the demixed state, without the amplification."""
    import numpy as np
    a, b = fields
    n = w.nodes
    last = checkpoints[-1]
    ref, ref_restart = {}, {}
    lat = P.Lattice(w.shape, tau=w.tau, G=w.G, storage="f64", device=0)
    try:
        lat.set_fields(a, b)
        done = 0
        for s in checkpoints:
            lat.step(s - done)
            done = s
            ref[s] = _moments(torch, lat, n)
        pop = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")
        lat.get_populations(pop)
        done = 0
        for s in restart:
            lat.step(s - done)
            done = s
            ref_restart[s] = _moments(torch, lat, n)
    finally:
        lat.close()

    sens = []
    lat = P.Lattice(w.shape, tau=w.tau, G=w.G, storage="f64", device=0)
    try:
        lat.set_fields(np.nextafter(a, np.inf), b)
        done = 0
        for s in checkpoints:
            lat.step(s - done)
            done = s
            sens.append(_error_row(torch, _moments(torch, lat, n), ref[s], step=s))
    finally:
        lat.close()

    out = {"f64_one_ulp": sens}
    for st in ("f32", "f16s"):
        lat = P.Lattice(w.shape, tau=w.tau, G=w.G, storage=st, device=0)
        try:
            lat.set_fields(a, b)
            done = 0
            rows = []
            for s in checkpoints:
                lat.step(s - done)
                done = s
                rows.append(_error_row(torch, _moments(torch, lat, n), ref[s], step=s))
            lat.set_populations(pop)
            done = 0
            rrows = []
            for s in restart:
                lat.step(s - done)
                done = s
                rrows.append(_error_row(torch, _moments(torch, lat, n), ref_restart[s], restart_step=last, steps=s))
            out[st] = {"trajectory": rows, "restart": rrows}
        finally:
            lat.close()
    # first step at which each form's max |drho| passes the 1e-3 target:
    # along the trajectory from the initial state, and after the restart
    for st in ("f32", "f16s"):
        out[st]["first_step_over_1e-3"] = first_step_over(P, torch, w, fields, st, None, limit=400)
        out[st]["restart_first_step_over_1e-3"] = first_step_over(P, torch, w, fields, st, pop, limit=10)
    del pop
    return out


def first_step_over(P, torch, w, fields, storage, start_pop=None, limit=400, bar=1e-3):
    """Step the float64 path and one reduced form side by side, from the
    initial fields or from the float64 populations ``start_pop``, and return
    the first step after which max |drho_k| exceeds ``bar`` (None if it does
    not within ``limit`` steps) with the error after every step."""
    a, b = fields
    n = w.nodes
    lats = [P.Lattice(w.shape, tau=w.tau, G=w.G, storage=st, device=0) for st in ("f64", storage)]
    errs = []
    first = None
    try:
        for lat in lats:
            if start_pop is None:
                lat.set_fields(a, b)
            else:
                lat.set_populations(start_pop)
        for s in range(1, limit + 1):
            for lat in lats:
                lat.step(1)
            ref = _moments(torch, lats[0], n)
            got = _moments(torch, lats[1], n)
            e = float(torch.maximum((got[0] - ref[0]).abs(), (got[1] - ref[1]).abs()).max())
            errs.append(e)
            if e > bar:
                first = s
                break
    finally:
        for lat in lats:
            lat.close()
    return {"bar": bar, "first_step": first, "limit": limit, "max_drho_per_step": [float(f"{e:.3e}") for e in errs]
            if len(errs) <= 20 else [float(f"{e:.3e}") for e in errs[-5:]], "steps_run": len(errs)}


def oracle_sample(name, w, planes, steps, make_state, advance):
    """Time an FP64 oracle on the first ``planes`` z-planes of a workload's
    initial state (bounded CPU time); returns a cpu_baseline object."""
    nz, ny, nx = w.shape
    planes = min(nz, planes)
    f = make_state((planes, ny, nx))
    t0 = time.perf_counter()
    advance(f, steps)
    dt = time.perf_counter() - t0
    nodes = planes * ny * nx
    return {
        "value": nodes * steps / dt / 1e9,
        "unit": "GLUPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{steps} steps of the float64 NumPy {name} oracle on a {nx}x{ny}x{planes} slab of the {w.name} "
                  f"initial state ({nodes} of {w.nodes} nodes, {dt:.1f} s; NumPy elementwise work is "
                  f"single-threaded)",
    }


def single_fluid_run(P, torch, synth, steps: int = 200, warmup: int = 10, cpu: bool = False):
    """The single-fluid fused step (the paper's case 1) on 256^3 in float32
    and float64: GLUPS and the fraction of the HBM roofline at 19 values read
    and 19 written per node."""
    out = {"workload": "case1_256", "lattice": [256, 256, 256],
           "paper_context": "2.011 GLUPS: one fluid, fused step, 256^3, single precision, one V100 (Table 1)"}
    for st in ("f32", "f64"):
        w = synth.WORKLOADS[f"case1_256_{st}"]
        rho, _ = synth.fluid_fields(w.shape, w.amp, w.seed)
        lat = P.SingleFluid(w.shape, tau=w.tau[0], storage=w.storage, device=0)
        try:
            lat.set_fields(rho.reshape(-1))
            lat.step(warmup)
            torch.cuda.synchronize()
            (m0, *_), _ = lat.totals()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            lat.step(steps)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            (m1, *_), nonfinite = lat.totals()
        finally:
            lat.close()
        glups = w.nodes / (ms * 1e-3) / 1e9
        bpl = 19 * 2 * BYTES_PER_VALUE[st]
        out[st] = {"glups": round(glups, 4), "ms_per_step": round(ms, 4), "bytes_per_lup": bpl,
                   "hbm_frac": round(bpl * glups / HBM_PEAK_GBS, 4), "mass_drift": abs(m1 - m0) / m0,
                   **traffic_fields(w.name, "k1_step", ms),
                   "nonfinite": nonfinite}
    if cpu:
        from oracle import lb_single as S

        w = synth.WORKLOADS["case1_256_f64"]
        rho, _ = synth.fluid_fields(w.shape, w.amp, w.seed)
        out["cpu_baseline"] = oracle_sample("single-fluid", w, 64, 4,
                                            lambda sh: S.init_equilibrium(rho[:sh[0]]),
                                            lambda f, n: S.step(f, w.tau[0], n=n))
    return out


def spheres_run(P, torch, synth, steps: int = 100, warmup: int = 10):
    """The 512^3 float32 lattice with 2000 fixed spheres of radius 5.5 (the
    two-component step with bounce-back at solid nodes): GLUPS over all
    nodes and over fluid nodes, mass drift."""
    w = synth.WORKLOADS["spheres512_f32"]
    a, b = synth.fluid_fields(w.shape, w.amp, w.seed)
    centres = synth.sphere_centres(w.shape, w.spheres, w.radius, w.sphere_seed)
    solid = synth.solid_mask(w.shape, centres, w.radius).reshape(-1)
    phi = float(solid.mean())
    r = time_form(P, torch, w, w.storage, steps, warmup, (a.reshape(-1), b.reshape(-1)), solid=solid)
    ms = r["event_ms"] / steps
    glups = w.nodes / (ms * 1e-3) / 1e9
    bpl = algorithmic_bytes_per_lup(w.storage)
    fused = r["kernels"].get("fused", {}).get("avg_ms")
    return {**traffic_fields(w.name, "fused", fused),
            "workload": w.name, "lattice": list(w.shape), "spheres": w.spheres, "solid_fraction": round(phi, 5),
            "glups": round(glups, 4), "fluid_glups": round(glups * (1.0 - phi), 4), "ms_per_step": round(ms, 4),
            "hbm_frac": round(bpl * glups / HBM_PEAK_GBS, 4), "mass_drift": r["mass_drift"],
            "nonfinite": r["nonfinite"]}


def particles_run(P, torch, synth, steps: int = 100, warmup: int = 10, cpu: bool = False):
    """Moving rigid spheres (radius 5.5, 2.2 times the fluid density) in the
    single-fluid step on 256^3: the paper's case-3 volume fractions 0.1%, 1%
    and 10%, float32 (and float64 at 10%).  GLUPS count every node; the
    overhead is the time per step over that of the same lattice without
    particles; hbm_frac_fluid prices the step at the fluid's own bytes (19
    populations each way and the owner word per node) against 8 TB/s, a
    lower bound of its traffic that leaves out the particle kernels'
    scattered accesses."""
    import numpy as np

    out = {"lattice": [256, 256, 256], "radius": 5.5, "fluid": "single fluid",
           "paper_context": "none like for like: the paper times particles in the two-fluid colour-gradient "
                            "model only (block cg_particles)"}
    base = {}
    for name in ("case3a_256_f32", "case3b_256_f32", "case3c_256_f32", "case3c_256_f64"):
        w = synth.WORKLOADS[name]
        rho, _ = synth.fluid_fields(w.shape, w.amp, w.seed)
        centres = synth.sphere_centres(w.shape, w.spheres, w.radius, w.sphere_seed)
        lat = P.SingleFluid(w.shape, tau=w.tau[0], storage=w.storage, device=0)
        try:
            lat.set_fields(rho.reshape(-1))
            if w.storage not in base:
                lat.step(warmup)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                lat.step(steps)
                e1.record()
                torch.cuda.synchronize()
                base[w.storage] = e0.elapsed_time(e1) / steps
                lat.set_fields(rho.reshape(-1))
            lat.set_particles(centres, w.radius, synth.particle_mass(w.radius))
            lat.step(warmup)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            lat.step(steps)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            _, nonfinite = lat.totals()
        finally:
            lat.close()
        phi = w.spheres * (4.0 / 3.0) * np.pi * w.radius ** 3 / w.nodes
        # fluid bytes per node: 19 populations read and written, plus the owner word
        bpl = 2 * 19 * (4 if w.storage == "f32" else 8) + 4
        if name == "case3c_256_f32":
            out["traffic_k1p_step"] = traffic_fields(name, "k1p_step")
            out["traffic_force_move"] = traffic_fields(name, "force_move")
        out[name] = {"spheres": w.spheres, "volume_fraction": round(phi, 5), "glups": round(w.nodes / (ms * 1e-3) / 1e9, 4),
                     "ms_per_step": round(ms, 4), "no_particles_ms_per_step": round(base[w.storage], 4),
                     "overhead": round(ms / base[w.storage] - 1.0, 4), "fluid_bytes_per_lup": bpl,
                     "hbm_frac_fluid": round(bpl * w.nodes / (ms * 1e-3) / 8e12, 4), "nonfinite": nonfinite}
    if cpu:
        from oracle import lb_particles as PT

        sh = (64, 64, 64)
        count = 38  # 10% of a 64^3 box in spheres of radius 5.5
        w = synth.WORKLOADS["case3c_256_f64"]
        centres = synth.sphere_centres(sh, count, w.radius, w.sphere_seed)
        rho, _ = synth.fluid_fields(sh, w.amp, w.seed)
        part = PT.Particles(w.radius, synth.particle_mass(w.radius), centres, None, None)
        f, owner = PT.init(rho, part)
        t0 = time.perf_counter()
        PT.step(f, w.tau[0], part, owner, n=2)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 64 ** 3 * 2 / dt / 1e9, "unit": "GLUPS", "cores": 1, "kind": "oracle",
                               "sample": f"2 steps of the float64 NumPy particle oracle on a 64^3 box with {count} "
                                         f"spheres of radius 5.5 (10%), {dt:.1f} s"}
    return out


def cg_particles_run(P, torch, synth, steps: int = 100, warmup: int = 10, cpu: bool = False):
    """The paper's case 3: moving rigid spheres (radius 5.5, 2.2 times the
    fluid density, at rest at the start) in the two immiscible fluids of
    case 2 (colour gradient, every node pure red or pure blue) on 256^3, at
    the volume fractions 0.1%, 1% and 10%, float32 (and float64 at 10%).
    GLUPS count every node.  The overhead is the time per step over that of
    the same fluid without particles (which runs on the tile-major layout);
    hbm_frac_fluid prices the step at the fluid's own bytes (38 populations
    each way and the owner word per node) against 8 TB/s."""
    import numpy as np

    out = {"lattice": [256, 256, 256], "radius": 5.5, "fluid": "colour gradient, two components",
           "paper_context": "34.6 / 37.6 / 56 ms per step (0.484 / 0.446 / 0.299 GLUPS) at 0.1 / 1 / 10% on one "
                            "V100, single precision (Sec. 5, particle table)"}
    base = {}
    for name in ("case3cg_a_256_f32", "case3cg_b_256_f32", "case3cg_c_256_f32", "case3cg_c_256_f64"):
        w = synth.WORKLOADS[name]
        r1, r2 = synth.colour_fields(w.shape, w.seed)
        centres = synth.sphere_centres(w.shape, w.spheres, w.radius, w.sphere_seed)
        lat = P.Lattice(w.shape, tau=w.tau, storage=w.storage, rho0=w.rho0, device=0, model="colour_gradient",
                        sigma=w.sigma, beta=w.beta)
        try:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            if w.storage not in base:
                lat.set_fields(r1.reshape(-1), r2.reshape(-1))
                lat.step(warmup)
                torch.cuda.synchronize()
                e0.record()
                lat.step(steps)
                e1.record()
                torch.cuda.synchronize()
                base[w.storage] = e0.elapsed_time(e1) / steps
            lat.set_fields(r1.reshape(-1), r2.reshape(-1))
            lat.set_particles(centres, w.radius, synth.particle_mass(w.radius))
            tot0, _ = lat.totals()
            lat.step(warmup)
            torch.cuda.synchronize()
            P.lb_timing(lat.ctx, True)
            e0.record()
            lat.step(steps)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            kernels = {}
            for sl in range(P.lb_timing_slots()):
                kms, cnt = P.lb_timing_read(lat.ctx, sl)
                if cnt:
                    kernels[P.lb_timing_name(sl)] = {"avg_ms": round(kms / cnt, 4), "launches": cnt}
            P.lb_timing(lat.ctx, False)
            tot1, nonfinite = lat.totals()
        finally:
            lat.close()
        phi = w.spheres * (4.0 / 3.0) * np.pi * w.radius ** 3 / w.nodes
        bpl = 2 * 2 * 19 * (4 if w.storage == "f32" else 8) + 4
        if name == "case3cg_c_256_f32":
            out["traffic_fused"] = traffic_fields(name, "fused", kernels.get("fused", {}).get("avg_ms"))
            out["traffic_force_move"] = traffic_fields(name, "force_move", kernels.get("part_force", {}).get("avg_ms"))
        out[name] = {"spheres": w.spheres, "volume_fraction": round(phi, 5),
                     "glups": round(w.nodes / (ms * 1e-3) / 1e9, 4), "ms_per_step": round(ms, 4),
                     "no_particles_ms_per_step": round(base[w.storage], 4),
                     "overhead": round(ms / base[w.storage] - 1.0, 4), "fluid_bytes_per_lup": bpl,
                     "hbm_frac_fluid": round(bpl * w.nodes / (ms * 1e-3) / 8e12, 4),
                     "kernels_timed_separately": kernels,
                     "mass_change": [(tot1[k] - tot0[k]) / tot0[k] for k in range(2)], "nonfinite": nonfinite}
    if cpu:
        from oracle import lb_cg_particles as CP
        from oracle import lb_particles as PT

        sh = (48, 48, 48)
        count = 16  # 10% of a 48^3 box in spheres of radius 5.5
        w = synth.WORKLOADS["case3cg_c_256_f64"]
        centres = synth.sphere_centres(sh, count, w.radius, w.sphere_seed)
        r1, r2 = synth.colour_fields(sh, w.seed)
        part = PT.Particles(w.radius, synth.particle_mass(w.radius), centres, None, None)
        f, owner = CP.init(r1, r2, part)
        p = CP.Params(w.tau, w.sigma, w.beta, w.rho0)
        t0 = time.perf_counter()
        CP.step(f, p, part, owner, n=2)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 48 ** 3 * 2 / dt / 1e9, "unit": "GLUPS", "cores": 1, "kind": "oracle",
                               "sample": f"2 steps of the float64 NumPy colour-gradient particle oracle on a 48^3 box "
                                         f"with {count} spheres of radius 5.5 (10%), {dt:.1f} s"}
    return out


def colour_gradient_run(P, torch, synth, steps: int = 200, warmup: int = 10, cpu: bool = False):
    """The colour-gradient step (the paper's case 2, two immiscible fluids) on
    256^3 in float32 and float64: GLUPS and the fraction of the HBM roofline
    at 38 values read and 38 written per node."""
    out = {"workload": "case2_256", "lattice": [256, 256, 256],
           "paper_context": "0.601 GLUPS: colour gradient, two-pass step, 256^3, single precision, one V100 (Sec. 5, "
                            "two-fluid table)"}
    for st in ("f32", "f64"):
        w = synth.WORKLOADS[f"case2_256_{st}"]
        r1, r2 = synth.colour_fields(w.shape, w.seed)
        lat = P.Lattice(w.shape, tau=w.tau, storage=w.storage, device=0, model="colour_gradient", sigma=w.sigma,
                        beta=w.beta)
        try:
            lat.set_fields(r1.reshape(-1), r2.reshape(-1))
            (a0, b0, *_), _ = lat.totals()  # before the warmup, which then takes the reorder into the step's order
            lat.step(warmup)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            lat.step(steps)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            (a1, b1, *_), nonfinite = lat.totals()
        finally:
            lat.close()
        glups = w.nodes / (ms * 1e-3) / 1e9
        bpl = 2 * 19 * 2 * BYTES_PER_VALUE[st]
        out[st] = {"glups": round(glups, 4), "ms_per_step": round(ms, 4), "bytes_per_lup": bpl,
                   "hbm_frac": round(bpl * glups / HBM_PEAK_GBS, 4), **traffic_fields(w.name, "fused", ms),
                   "mass_drift": max(abs(a1 - a0) / a0, abs(b1 - b0) / b0), "nonfinite": nonfinite}
    if cpu:
        from oracle import lb_cg as CG

        w = synth.WORKLOADS["case2_256_f64"]
        r1, r2 = synth.colour_fields(w.shape, w.seed)
        p = CG.Params(w.tau, w.sigma, w.beta)
        out["cpu_baseline"] = oracle_sample("colour-gradient", w, 32, 3,
                                            lambda sh: CG.init_equilibrium(r1[:sh[0]], r2[:sh[0]]),
                                            lambda f, n: CG.step(f, p, n=n))
    return out


def adjoint_run(P, torch, synth, every: int = 50, fd: bool = True):
    """Forward (with checkpoint saves) and backward (recompute + adjoint) of
    J = sum (rho_A(T) - target)^2 on the 128^3, 500-step gradient workload,
    in float32 and in float64 storage.

    * ratio: backward (seeding, restores, recomputation, adjoint steps,
      read-out) over forward (the steps and checkpoint saves), both device
      time; also over the plain 500 forward steps alone.
    * float32 against float64: the float32 adjoint's dJ/drho_A(0) at 16
      sites (seed 5) and over the whole field, and its dJ/dG, relative to the
      float64 adjoint.
    * float64 against differences: fourth-order central differences of the
      float64 forward (h = 2e-5, objective summed exactly) at the same 16
      sites and for G; the error of each site relative to the largest sampled
      |gradient| (the normalisation of the 1e-6 target) and to its own value.
    """
    import math

    import numpy as np

    from paper_2112_08264_amd import autograd as AG

    w = synth.WORKLOADS["adjoint128_f32"]
    a, b = synth.fluid_fields(w.shape, w.amp, w.seed)
    target_np = synth.smooth_target(w.shape, 4)
    target = torch.tensor(target_np, device="cuda")
    sites = synth.sample_sites(w.shape, 16, 5)

    def gradient(storage):
        spec = AG.Spec(shape=w.shape, tau=w.tau, steps=w.steps, every=every, storage=storage)
        ra = torch.tensor(a, device="cuda", requires_grad=True)
        rb = torch.tensor(b, device="cuda")
        G = torch.tensor(w.G, dtype=torch.float64, requires_grad=True)
        out = AG.final_density(ra, G, rb, spec)
        J = ((out - target) ** 2).sum()
        J.backward()
        return float(J), ra.grad.detach().cpu().numpy(), float(G.grad)

    def plain_forward_ms(storage):
        lat = P.Lattice(w.shape, tau=w.tau, G=w.G, storage=storage, device=0)
        try:
            lat.set_fields(a.reshape(-1).copy(), b.reshape(-1).copy())
            lat.step(10)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            lat.step(w.steps)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1)
        finally:
            lat.close()

    forms = {}
    grads = {}
    for storage in ("f32", "f64"):
        gradient(storage)  # warm-up (allocations, code objects)
        J, ga, dG = gradient(storage)
        fwd, bwd = AG.timings.forward_ms, AG.timings.backward_ms
        plain = plain_forward_ms(storage)
        grads[storage] = (J, ga, dG)
        forms[storage] = {"forward_ms": round(fwd, 3), "backward_ms": round(bwd, 3), "ratio": round(bwd / fwd, 3),
                          "plain_forward_ms": round(plain, 3), "ratio_to_plain_forward": round(bwd / plain, 3),
                          "J": J, "dJ_dG": dG, "max_abs_dJ_drhoA0": float(np.max(np.abs(ga)))}
    J32, g32, dG32 = grads["f32"]
    J64, g64, dG64 = grads["f64"]
    at = [(int(x), int(y), int(z)) for x, y, z in sites]
    s64 = np.array([g64[z, y, x] for x, y, z in at])
    s32 = np.array([g32[z, y, x] for x, y, z in at])
    f32_vs_f64 = {"sites": 16, "site_seed": 5,
                  "max_site_error_over_max_site_gradient": float(np.max(np.abs(s32 - s64)) / np.max(np.abs(s64))),
                  "max_site_relative_error": float(np.max(np.abs(s32 - s64) / np.abs(s64))),
                  "field_max_error_over_max_gradient": float(np.max(np.abs(g32 - g64)) / np.max(np.abs(g64))),
                  "dJ_dG_relative_error": abs(dG32 - dG64) / abs(dG64),
                  "J_relative_error": abs(J32 - J64) / abs(J64)}
    out = {"workload": w.name, "steps": w.steps, "checkpoint_every": every, "forms": forms,
           "f32_vs_f64_adjoint": f32_vs_f64,
           "traffic_adj_local": traffic_fields(w.name, "adj_local"), "traffic_adj_r": traffic_fields(w.name, "adj_r"),
           # the float32 form is the workload's own storage; kept at the top level for continuity
           "forward_ms": forms["f32"]["forward_ms"], "backward_ms": forms["f32"]["backward_ms"],
           "ratio": forms["f32"]["ratio"]}
    if not fd:
        return out
    tt = target.view(-1)

    def J_of(ra, G=w.G):
        lat = P.Lattice(w.shape, tau=w.tau, G=G, storage="f64", device=0)
        try:
            lat.set_fields(ra.reshape(-1).copy(), b.reshape(-1).copy())
            lat.step(w.steps)
            r = torch.empty(ra.size, dtype=torch.float64, device="cuda")
            lat.moments(rho_a=r)
        finally:
            lat.close()
        return math.fsum(((r - tt) ** 2).cpu().numpy())

    def d4(f, h):
        return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)

    rows = []
    for x, y, z in at:
        def f(eps, x=x, y=y, z=z):
            ap = a.copy()
            ap[z, y, x] += eps
            return J_of(ap)
        rows.append((d4(f, 2e-5), float(g64[z, y, x])))
    fdG = d4(lambda eps: J_of(a, w.G + eps), 1e-5)
    fdv = np.array([r[0] for r in rows])
    adj = np.array([r[1] for r in rows])
    err = np.abs(fdv - adj)
    out["f64_vs_differences"] = {
        "sites": 16, "h": 2e-5, "order": 4,
        "max_site_error_over_max_site_gradient": float(np.max(err) / np.max(np.abs(fdv))),
        "median_site_error_over_max_site_gradient": float(np.median(err) / np.max(np.abs(fdv))),
        "max_site_relative_error": float(np.max(err / np.abs(fdv))),
        "median_site_relative_error": float(np.median(err / np.abs(fdv))),
        "dJ_dG_relative_error": abs(fdG - dG64) / abs(fdG),
        "max_abs_site_gradient": float(np.max(np.abs(fdv))),
        "min_abs_site_gradient": float(np.min(np.abs(fdv)))}
    return out


def copy_calibration(torch, nbytes: int = 2 << 30, reps: int = 5):
    """Plain device-to-device copy of a known size: the reference kernel for
    scaling rocprofv3's FETCH_SIZE / WRITE_SIZE and for attainable bandwidth."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "ms": ms,
            "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}


def attainable_bandwidth(torch, nbytes: int = 2 << 30, reps: int = 10):
    """Best read-plus-write bandwidth of plain streaming kernels over 2 GiB:
    torch's device copy, and elementwise scaling by 1 in float64 and float32."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    s32, d32 = src.view(torch.float32), dst.view(torch.float32)
    ops = {"copy": lambda: dst.copy_(src), "scale_f64": lambda: torch.mul(src, 1.0, out=dst),
           "scale_f32": lambda: torch.mul(s32, 1.0, out=d32)}
    best = (0.0, None)
    for name, fn in ops.items():
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        gbs = 2 * nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
        best = max(best, (gbs, name))
    return {"gbs": round(best[0], 1), "kernel": best[1]}


def cpu_baseline(w, fields_fn):
    """The FP64 oracle on the host, on a slab of the same lattice (bounded CPU time)."""
    import numpy as np

    from oracle import lb_oracle as O

    nz, ny, nx = w.shape
    planes = min(nz, 96)
    steps = 4
    a, b = fields_fn()
    a = np.ascontiguousarray(a.reshape(w.shape)[:planes])
    b = np.ascontiguousarray(b.reshape(w.shape)[:planes])
    f = O.init_equilibrium(a, b)
    p = O.Params(w.tau, w.G)
    t0 = time.perf_counter()
    f = O.step(f, p, n=steps)
    dt = time.perf_counter() - t0
    nodes = planes * ny * nx
    return {
        "value": nodes * steps / dt / 1e9,
        "unit": "GLUPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{steps} steps of the float64 NumPy oracle on a {nx}x{ny}x{planes} slab of the {w.name} "
                  f"initial state ({nodes} of {w.nodes} nodes, {dt:.1f} s; NumPy elementwise work is "
                  f"single-threaded; host has {os.cpu_count()} logical CPUs)",
    }


# Kernels whose HBM traffic is measured (rocprofv3 FETCH_SIZE / WRITE_SIZE):
# target -> (workload, {key in profiles/traffic.json: kernel symbol substring}).
PROFILE_TARGETS = {
    "sc_f64": ("spinodal256_f64", {"fused": "k_fused_pair<"}),
    "sc_f32": ("spinodal256_f32", {"fused": "k_fused<"}),
    "sc_f16s": ("spinodal256_f16s", {"fused": "k_fused<"}),
    "cg_f32": ("case2_256_f32", {"fused": "k_fused_pair<"}),
    "cg_f64": ("case2_256_f64", {"fused": "k_fused_pair<"}),
    "single_f32": ("case1_256_f32", {"k1_step": "k1_step<"}),
    "single_f64": ("case1_256_f64", {"k1_step": "k1_step<"}),
    "spheres_f32": ("spheres512_f32", {"fused": "k_fused<"}),
    "adjoint_f32": ("adjoint128_f32", {"adj_local": "k_adj_local<", "adj_r": "k_adj_r_march<"}),
    "particles_f32": ("case3c_256_f32", {"k1p_step": "k1p_step<", "force_move": "kp_force_move<"}),
    "cgp_f32": ("case3cg_c_256_f32", {"fused": "k_fused_pair<", "force_move": "kp_force_move<"}),
}


def profile_target(P, torch, synth, name: str, steps: int, warmup: int) -> dict:
    """Run only the kernels of one PROFILE_TARGETS entry, ``warmup`` then
    ``steps`` steps (the command rocprofv3 counts HBM bytes on)."""
    import numpy as np

    wname, _ = PROFILE_TARGETS[name]
    w = synth.WORKLOADS[wname]
    t0 = time.perf_counter()
    if name.startswith("single"):
        rho, _ = synth.fluid_fields(w.shape, w.amp, w.seed)
        with P.SingleFluid(w.shape, tau=w.tau[0], storage=w.storage, device=0) as lat:
            lat.set_fields(rho.reshape(-1))
            lat.step(warmup + steps)
            torch.cuda.synchronize()
    elif name.startswith("particles"):
        rho, _ = synth.fluid_fields(w.shape, w.amp, w.seed)
        centres = synth.sphere_centres(w.shape, w.spheres, w.radius, w.sphere_seed)
        with P.SingleFluid(w.shape, tau=w.tau[0], storage=w.storage, device=0) as lat:
            lat.set_fields(rho.reshape(-1))
            lat.set_particles(centres, w.radius, synth.particle_mass(w.radius))
            lat.step(warmup + steps)
            torch.cuda.synchronize()
    elif name.startswith("cgp"):
        r1, r2 = synth.colour_fields(w.shape, w.seed)
        centres = synth.sphere_centres(w.shape, w.spheres, w.radius, w.sphere_seed)
        with P.Lattice(w.shape, tau=w.tau, storage=w.storage, rho0=w.rho0, device=0, model="colour_gradient",
                       sigma=w.sigma, beta=w.beta) as lat:
            lat.set_fields(r1.reshape(-1), r2.reshape(-1))
            lat.set_particles(centres, w.radius, synth.particle_mass(w.radius))
            lat.step(warmup + steps)
            torch.cuda.synchronize()
    elif name.startswith("cg"):
        r1, r2 = synth.colour_fields(w.shape, w.seed)
        with P.Lattice(w.shape, tau=w.tau, storage=w.storage, device=0, model="colour_gradient", sigma=w.sigma,
                       beta=w.beta) as lat:
            lat.set_fields(r1.reshape(-1), r2.reshape(-1))
            lat.step(warmup + steps)
            torch.cuda.synchronize()
    elif name.startswith("adjoint"):
        from paper_2112_08264_amd import autograd as AG

        a, b = synth.fluid_fields(w.shape, w.amp, w.seed)
        spec = AG.Spec(shape=w.shape, tau=w.tau, steps=warmup + steps, every=warmup + steps, storage=w.storage)
        ra = torch.tensor(a, device="cuda", requires_grad=True)
        G = torch.tensor(w.G, dtype=torch.float64, requires_grad=True)
        out = AG.final_density(ra, G, torch.tensor(b, device="cuda"), spec)
        ((out - 1.0) ** 2).sum().backward()
        torch.cuda.synchronize()
    else:
        a, b = synth.fluid_fields(w.shape, w.amp, w.seed)
        solid = None
        if w.spheres:
            centres = synth.sphere_centres(w.shape, w.spheres, w.radius, w.sphere_seed)
            solid = synth.solid_mask(w.shape, centres, w.radius).reshape(-1)
        with P.Lattice(w.shape, tau=w.tau, G=w.G, storage=w.storage, device=0) as lat:
            lat.set_fields(a.reshape(-1), b.reshape(-1), None, solid)
            lat.totals()
            lat.step(warmup + steps)
            torch.cuda.synchronize()
    return {"profile_target": name, "workload": wname, "steps": steps, "warmup": warmup,
            "seconds": round(time.perf_counter() - t0, 2), "np": np.__version__}


def link_count(synth, wname: str) -> int:
    """Links (particle node, direction with a fluid neighbour) of a particle
    workload's initial positions: the unit of the link pass's algorithmic
    bytes."""
    import numpy as np

    w = synth.WORKLOADS[wname]
    centres = synth.sphere_centres(w.shape, w.spheres, w.radius, w.sphere_seed)
    solid = synth.solid_mask(w.shape, centres, w.radius).astype(bool)
    dirs = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
            if 0 < abs(dx) + abs(dy) + abs(dz) <= 2]
    n = 0
    for dx, dy, dz in dirs:
        nb = np.roll(solid, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
        n += int(np.count_nonzero(solid & ~nb))
    return n


def algorithmic_bytes(synth, target: str, key: str):
    """Algorithmic HBM bytes of one launch of a measured kernel: every value
    the kernel must read and write once (None where that is not defined)."""
    wname, _ = PROFILE_TARGETS[target]
    w = synth.WORKLOADS[wname]
    es = BYTES_PER_VALUE[w.storage]
    if key == "fused":
        if target.startswith("cgp"):
            return w.nodes * (2 * 2 * 19 * es + 4)  # populations both ways and the owner word
        return w.nodes * algorithmic_bytes_per_lup(w.storage)
    if key == "k1_step":
        return w.nodes * 2 * 19 * es
    if key == "k1p_step":
        return w.nodes * (2 * 19 * es + 4)
    if key == "adj_local":
        # lambda (P) 38 values pulled and 38 written, r (2) pulled, the moment record (10) read, W (6) written
        return w.nodes * (38 + 38 + 2 + 10 + 6) * 4
    if key == "adj_r":
        return w.nodes * (6 + 2) * 4  # W read once, r written
    if key == "force_move":
        comps = 2 if target.startswith("cgp") else 1
        # per link and component: the pushed value read, the bounce-back stored, the slot cleared, the
        # recorded float64 density read; per link: the neighbour's owner word
        return link_count(synth, wname) * (comps * (3 * es + 8) + 4)
    return None


def traffic_from_profile(kernel: str, workload: str, lups_per_launch: int):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        ent = data[workload][kernel]
    except (KeyError, ValueError):
        return None
    if ent.get("source_digest") != source_digest():
        return None
    return ent.get("bytes_per_launch")


def write_traffic(prof_dir: str, target: str = "sc_f64") -> dict:
    """Turn two rocprofv3 counter runs of ``bench.py --profile-target TARGET``
    (FETCH_SIZE, then WRITE_SIZE, under DIR/pmc_<COUNTER>/) and two of
    ``--calibrate`` (DIR/cal_<COUNTER>/, may be shared by several targets)
    into HBM bytes per launch of the target's kernels, scaled by what the
    counters read for the 2 GiB copy, and record them in
    profiles/traffic.json under the workload and the current kernel source
    digest."""
    import csv

    import synth

    def rows(sub, prefix):
        path = os.path.join(prof_dir, sub, f"{prefix}_counter_collection.csv")
        with open(path, newline="") as fh:
            return list(csv.DictReader(fh))

    def per_kernel(rs):
        acc = {}
        for r in rs:
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return acc

    wname, keys = PROFILE_TARGETS[target]
    copy_bytes = 2 << 30
    scale = {}
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        cal = per_kernel(rows(f"cal_{counter}", "cal"))
        copy_kib = [v for k, vs in cal.items() if "copyBuffer" in k for v in vs]
        scale[counter] = copy_bytes / (max(copy_kib) * 1024.0)
    measured = {c: per_kernel(rows(os.path.join(target, f"pmc_{c}"), "pmc")) for c in ("FETCH_SIZE", "WRITE_SIZE")}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    entries = {}
    for key, sub in keys.items():
        out = {}
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            ker = measured[counter]
            names = [k for k in ker if sub in k]
            name = max(names, key=lambda k: sum(ker[k]))
            kib = sum(ker[name]) / len(ker[name])
            out[counter] = {"kernel": name, "kib": kib, "bytes": kib * 1024.0 * scale[counter],
                            "dispatches": len(ker[name])}
        total = out["FETCH_SIZE"]["bytes"] + out["WRITE_SIZE"]["bytes"]
        alg = algorithmic_bytes(synth, target, key)
        entry = {
            "bytes_per_launch": int(round(total)),
            "read_bytes_per_launch": int(round(out["FETCH_SIZE"]["bytes"])),
            "write_bytes_per_launch": int(round(out["WRITE_SIZE"]["bytes"])),
            "fetch_size_kib": out["FETCH_SIZE"]["kib"],
            "write_size_kib": out["WRITE_SIZE"]["kib"],
            "read_scale": scale["FETCH_SIZE"],
            "write_scale": scale["WRITE_SIZE"],
            "algorithmic_bytes_per_launch": alg,
            "ratio_to_algorithmic": None if not alg else total / alg,
            "kernel_symbol": out["FETCH_SIZE"]["kernel"],
            "dispatches": [out["FETCH_SIZE"]["dispatches"], out["WRITE_SIZE"]["dispatches"]],
            "profile_target": target,
            "source_digest": source_digest(),
        }
        data.setdefault(wname, {})[key] = entry
        entries[key] = entry
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1)
        fh.write("\n")
    return entries


def traffic_entry(workload: str, key: str):
    """The committed counter entry of one kernel, if it was taken on the
    current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        ent = json.load(open(path))[workload][key]
    except (KeyError, ValueError):
        return None
    return ent if ent.get("source_digest") == source_digest() else None


def traffic_fields(workload: str, key: str, avg_ms=None) -> dict:
    """Measured HBM bytes of a kernel next to its algorithmic bytes, and the
    achieved fraction of 8 TB/s at its average launch time."""
    ent = traffic_entry(workload, key)
    if ent is None:
        return {"traffic": None}
    out = {"traffic": ent["bytes_per_launch"], "traffic_ratio_to_algorithmic": ent["ratio_to_algorithmic"],
           "algorithmic_bytes_per_launch": ent["algorithmic_bytes_per_launch"]}
    if avg_ms and ent["algorithmic_bytes_per_launch"]:
        out["frac"] = round(ent["algorithmic_bytes_per_launch"] / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        out["measured_bytes_frac"] = round(ent["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="spinodal256_f64")
    ap.add_argument("--form-steps", type=int, default=200, help="timed steps of the float32 / float16 forms")
    ap.add_argument("--no-forms", action="store_true", help="skip the float32 / float16-shifted forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward timing")
    ap.add_argument("--no-adjoint-fd", action="store_true",
                    help="skip the float64 finite-difference table of the adjoint block (about 70 forward runs)")
    ap.add_argument("--no-single", action="store_true", help="skip the single-fluid (case 1) timing")
    ap.add_argument("--no-cg", action="store_true", help="skip the colour-gradient (case 2) timing")
    ap.add_argument("--no-particles", action="store_true", help="skip the moving-particle (case 3 fractions) timing")
    ap.add_argument("--no-spheres", action="store_true", help="skip the 512^3 fixed-sphere timing")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the reduced-precision error report")
    ap.add_argument("--kernel", default="auto", choices=["auto", "fused", "two_pass", "fused_staged"])
    ap.add_argument("--calibrate", action="store_true",
                    help="only time a plain device copy of 2 GiB (reference for HBM counters and bandwidth)")
    ap.add_argument("--write-traffic", metavar="DIR",
                    help="no GPU: read rocprofv3 counter CSVs under DIR (cal_<COUNTER>/ and "
                         "<target>/pmc_<COUNTER>/ for FETCH_SIZE, WRITE_SIZE) and record the HBM bytes per launch "
                         "of the --profile-target's kernels in profiles/traffic.json")
    ap.add_argument("--profile-target", choices=sorted(PROFILE_TARGETS),
                    help="run only this target's kernels for --warmup + --steps steps (for rocprofv3 counters)")
    args = ap.parse_args(argv)

    if args.write_traffic:
        print(json.dumps(write_traffic(args.write_traffic, args.profile_target or "sc_f64")), flush=True)
        return 0

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        return 2

    import torch

    import paper_2112_08264_amd as P
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    P.library()  # raises if liblb.so is missing: there is no fallback
    torch.cuda.set_device(0)
    if args.calibrate:
        print(json.dumps(copy_calibration(torch)), flush=True)
        return 0
    if args.profile_target:
        print(json.dumps(profile_target(P, torch, synth, args.profile_target, args.steps, args.warmup)), flush=True)
        return 0
    w = synth.WORKLOADS[args.workload]
    log(f"bench: workload {w.name} {w.shape} storage {w.storage}; generating inputs")
    a, b = synth.fluid_fields(w.shape, w.amp, w.seed)
    fields = (a.reshape(-1), b.reshape(-1))
    solid = None
    solid_fraction = 0.0
    if w.spheres:
        centres = synth.sphere_centres(w.shape, w.spheres, w.radius, w.sphere_seed)
        solid = synth.solid_mask(w.shape, centres, w.radius).reshape(-1)
        solid_fraction = float(solid.mean())
        log(f"bench: {w.spheres} spheres of radius {w.radius}, solid fraction {solid_fraction:.4f}")

    log(f"bench: {args.warmup} warmup + {args.steps} timed steps")
    main_run = time_form(P, torch, w, w.storage, args.steps, args.warmup, fields, kernel=args.kernel, solid=solid,
                         repeats=3)
    ms_step = main_run["event_ms"] / args.steps
    glups = w.nodes / (ms_step * 1e-3) / 1e9
    bpl = algorithmic_bytes_per_lup(w.storage)
    log(f"bench: {ms_step:.3f} ms/step, {glups:.3f} GLUPS, kernels {main_run['kernels']}")

    # dominant kernel: the one with the largest summed time
    kernels = main_run["kernels"]
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    dom_ms = kernels[dom]["avg_ms"]
    achieved = bpl * w.nodes / (dom_ms * 1e-3) / 1e9
    traffic = traffic_from_profile(dom, w.name, w.nodes)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "algorithmic_bytes_per_lup": bpl, "lups_per_launch": w.nodes}
    # attainable bandwidth on this device: the best plain streaming kernel over 2 GiB
    att = attainable_bandwidth(torch)
    copy_bw = {"gbs": att["gbs"], "kernel": att["kernel"], "frac_of_peak": round(att["gbs"] / HBM_PEAK_GBS, 4),
               "step_frac_of_copy": round(achieved / att["gbs"], 4)}

    forms = {}
    if not args.no_forms and solid is None:
        for st in ("f32", "f16s"):
            if st == w.storage:
                continue
            log(f"bench: form {st}, {args.form_steps} steps")
            r = time_form(P, torch, w, st, args.form_steps, 10, fields, kernel=args.kernel)
            ms = r["event_ms"] / args.form_steps
            g = w.nodes / (ms * 1e-3) / 1e9
            forms[st] = {"glups": round(g, 4), "ms_per_step": round(ms, 4),
                         "step_hbm_frac": round(algorithmic_bytes_per_lup(st) * g / HBM_PEAK_GBS, 4),
                         "vs_f64": round(g / glups, 3) if w.storage == "f64" else None,
                         "nonfinite": r["nonfinite"], "kernels": r["kernels"],
                         **traffic_fields(f"{w.name.rsplit('_', 1)[0]}_{st}", "fused",
                                          r["kernels"].get("fused", {}).get("avg_ms"))}

    accuracy = None
    if not args.no_accuracy and solid is None and w.storage == "f64":
        log("bench: float32 / float16-shifted error against the float64 path")
        accuracy = accuracy_run(P, torch, w, fields)
        for st in ("f32", "f16s"):
            if st in forms:
                forms[st]["error_vs_f64"] = accuracy[st]["trajectory"]
                forms[st]["error_vs_f64_restart"] = accuracy[st]["restart"]
                forms[st]["first_step_over_1e-3"] = accuracy[st]["first_step_over_1e-3"]
                forms[st]["restart_first_step_over_1e-3"] = accuracy[st]["restart_first_step_over_1e-3"]

    adjoint = None
    if not args.no_adjoint:
        log("bench: adjoint 128^3, float32 and float64, 500 steps, checkpoint every 50")
        adjoint = adjoint_run(P, torch, synth, fd=not args.no_adjoint_fd)
        log(f"bench: adjoint {adjoint}")

    single = None
    if not args.no_single:
        log("bench: single fluid (case 1) 256^3, float32 and float64")
        single = single_fluid_run(P, torch, synth, cpu=not args.no_cpu_baseline)
        log(f"bench: single fluid {single}")

    cg = None
    if not args.no_cg:
        log("bench: colour gradient (case 2) 256^3, float32 and float64")
        cg = colour_gradient_run(P, torch, synth, cpu=not args.no_cpu_baseline)
        log(f"bench: colour gradient {cg}")

    spheres = None
    if not args.no_spheres and w.name != "spheres512_f32":
        log("bench: 512^3 float32 with 2000 fixed spheres")
        spheres = spheres_run(P, torch, synth)
        log(f"bench: spheres {spheres}")

    particles = None
    if not args.no_particles:
        log("bench: moving particles 256^3, 0.1 / 1 / 10% of the volume")
        particles = particles_run(P, torch, synth, cpu=not args.no_cpu_baseline)
        log(f"bench: particles {particles}")

    cg_particles = None
    if not args.no_particles:
        log("bench: moving particles in the colour-gradient fluid (case 3) 256^3, 0.1 / 1 / 10% of the volume")
        cg_particles = cg_particles_run(P, torch, synth, cpu=not args.no_cpu_baseline)
        log(f"bench: cg particles {cg_particles}")

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        cpu = cpu_baseline(w, lambda: (a, b))

    out = {
        "metric": METRIC,
        "value": round(glups, 4),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.storage,
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": list(reversed(w.shape)), "storage": w.storage,
                   "tau": list(w.tau), "G": w.G, "rho0": list(w.rho0), "noise": w.amp, "seed": w.seed,
                   "boundary": "periodic", "solid_spheres": w.spheres, "solid_fraction": round(solid_fraction, 5)},
        "step_hbm_frac": round(bpl * glups / HBM_PEAK_GBS, 4),
        # three more blocks of 300 steps after the timed region, for the median of repeated runs
        "repeat_ms_per_step": [round(v, 4) for v in main_run["repeat_ms_per_step"]],
        "repeat_median_ms_per_step": round(sorted(main_run["repeat_ms_per_step"])[1], 4)
        if len(main_run["repeat_ms_per_step"]) == 3 else None,
        "fluid_glups": round(glups * (1.0 - solid_fraction), 4),
        "roofline": roofline,
        "copy_bandwidth": copy_bw,
        "cpu_baseline": cpu,
        "forms": forms,
        "f64_one_ulp_sensitivity": None if accuracy is None else accuracy["f64_one_ulp"],
        "adjoint_forward_ratio": None if adjoint is None else adjoint["ratio"],
        "adjoint_forward_ratio_f64": None if adjoint is None else adjoint["forms"]["f64"]["ratio"],
        "adjoint": adjoint,
        "single_fluid": single,
        "colour_gradient": cg,
        "spheres": spheres,
        "particles": particles,
        "cg_particles": cg_particles,
        "mass_drift": main_run["mass_drift"],
        "nonfinite": main_run["nonfinite"],
        "wall_ms": round(main_run["wall_ms"], 2),
        "kernel": args.kernel,
        "kernel_source_digest": source_digest(),
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
