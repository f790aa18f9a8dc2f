"""Benchmark of the fused BSSN RHS + RK4 path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload bl2-384-o8]

One "step" is one classical RK4 step (four fused stage launches) over the
whole grid.  The timed region covers exactly K steps with inputs resident in
HBM, bracketed by device synchronisations; HIP events recorded on the launch
stream around every stage give the average kernel duration used for the
roofline.  Prints ONE JSON line.

The default run's headline is the largest single-grid workload, two
Brill-Lindquist punctures on 384^3 + 5 ghosts with 8th-order differences:
`value` is its FP64 rate, `mixed` the mixed-precision one, `roofline` the
FP64 stage kernel against 8 TB/s (and against a 4 GiB device copy timed in
the same run), `cpu_baseline` the FP64 oracle on the host cores (model,
thread count, one-thread rate).  `workloads` adds the 256^3 and 128^3
grids (FP64 and mixed; on 128^3 also the constraint norms after 100 RK4
steps) and the 256 uneven patches (batched against one launch per patch);
`extras` times the steps around the path on the 128^3 grid; `accuracy`
runs the 384^3 (50 steps) and 256^3 (200 steps) workloads in FP64 and in
mixed precision and compares fields and constraint norms.

Profiling support (the summaries under profiles/ are made this way):
    rocprofv3 --kernel-trace --stats --output-format csv -d D -o run \
        -- python bench.py                      # kernel durations
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d D -o run \
        -- python bench.py --steps 2 --warmup 0 --no-cpu-baseline \
           --no-mixed --calibrate-copy          # then WRITE_SIZE alike
    python bench.py --summarize-profile D1 D2 ... > profiles/<name>.txt
--calibrate-copy ends the run with three plain device-to-device copies of
1 GiB, so the HBM byte counters can be scaled by what they read for a copy
of known size.  The roofline's `traffic` is taken from
profiles/traffic_<kernel>_<workload>.txt when the kernel sources still
hash to the value recorded there, else it is null.

Algorithmic HBM bytes per interior point (25 FP64 slots = 200 B per state):
stage 0: read u_n, write acc and u_out = 600 B; stages 1, 2: read u_s, u_n,
acc, write acc, u_out = 1000 B; stage 3: read u_s, acc, write u_out = 600 B;
3200 B per point-step.  Mixed precision keeps the state in FP64, so its bytes
are the same.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

STAGE_BYTES = (600, 1000, 1000, 600)
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

WORKLOADS = {
    # name: (n, lo, hi, ghost, masses, centres, order, dt, description)
    "noise32": (32, -1.6, 1.6, 3, None, None, 4, 0.025,
           "32^3 + 3 ghosts periodic, Minkowski + 1e-8 noise, 4th order"),
    "bl1-128": (128, -8.0, 8.0, 3, (1.0,), ((0.0, 0.0, 0.0),), 4, 0.03125,
           "single Brill-Lindquist puncture M=1, 128^3 + 3 ghosts on "
           "[-8,8]^3, static boundary, 4th-order FD, KO eps=0.1, RK4 "
           "dt=0.03125"),
    "bl2-256": (256, -16.0, 16.0, 3, (0.5, 0.5), ((3.0, 0, 0), (-3.0, 0, 0)), 4,
           0.03125,
           "two Brill-Lindquist punctures m=0.5 at (+-3,0,0), 256^3 + 3 "
           "ghosts on [-16,16]^3, static boundary, 4th-order FD, RK4 "
           "dt=0.03125"),
    "patches256": (None, None, None, 3, None, None, 4, 0.03125,
           "256 uneven static patches, interiors U{24..96} per axis, "
           "3 ghosts, h=0.125, one Brill-Lindquist puncture each (mass "
           "U[0.3,1.0], seeded centre), 4th order, RK4 dt=0.03125"),
    "bl2-384-o8": (384, -24.0, 24.0, 5, (0.6, 0.4), ((4.0, 0, 0), (-4.0, 0, 0)), 8,
           0.03125,
           "two Brill-Lindquist punctures m=0.6/0.4 at (+-4,0,0), 384^3 "
           "+ 5 ghosts on [-24,24]^3, static boundary, 8th-order FD, RK4 "
           "dt=0.03125"),
}


def build_state(name):
    from paper_1111_3344_amd import inputs as I
    n, lo, hi, gh, masses, centres, order, dt, desc = WORKLOADS[name]
    if masses is None:
        g = I.cell_centred(n, lo, hi, gh, I.BC_PERIODIC)
        u = I.minkowski_noise(g)
    else:
        g = I.cell_centred(n, lo, hi, gh)
        u = I.brill_lindquist(g, masses, centres)
    return g, u, order, dt, desc


def time_gpu(B, torch, g, u_host, prm, dt, steps, warmup):
    """Returns (seconds for `steps` steps, per-stage mean kernel ms)."""
    du = torch.from_numpy(u_host).to("cuda")
    a, b, acc = du.clone(), du.clone(), torch.zeros_like(du)
    stream = torch.cuda.current_stream()
    bufs = [(du, du, a), (du, a, b), (du, b, a), (du, a, du)]
    for _ in range(warmup):
        for s, (un, us, uo) in enumerate(bufs):
            B.rk4_stage(g, prm, s, dt, un, us, acc, uo, stream)
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True)) for _ in range(4)]
          for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        for s, (un, us, uo) in enumerate(bufs):
            ev[k][s][0].record(stream)
            B.rk4_stage(g, prm, s, dt, un, us, acc, uo, stream)
            ev[k][s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_stage = [sum(ev[k][s][0].elapsed_time(ev[k][s][1])
                     for k in range(steps)) / steps for s in range(4)]
    del du, a, b, acc
    torch.cuda.empty_cache()
    return wall, per_stage


RADIATIVE_BYTES_PER_POINT = 600  # state of the point, right-hand side of
                                 # its inward neighbour, its own: 25 x 3 x 8


def time_radiative(B, torch, g, u_host, prm, reps=20, warmup=2):
    """bssn_radiative_rhs on the workload's grid, timed alone: the interior
    right-hand side comes from one bssn_rhs call, then reps boundary calls
    (each rewrites the ghost layers from the same interior) between HIP
    events on the launch stream."""
    du = torch.from_numpy(u_host).to("cuda")
    k = torch.zeros_like(du)
    stream = torch.cuda.current_stream()
    B.bssn_rhs(g, prm, du, k, stream)
    for _ in range(warmup):
        B.bssn_radiative_rhs(g, du, k, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        B.bssn_radiative_rhs(g, du, k, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    npts = 0
    for layer in range(1, g.ghost + 1):
        a = [g.n[i] + 2 * layer for i in range(3)]
        npts += (2 * a[0] * a[1] + 2 * a[0] * (a[2] - 2) +
                 2 * (a[1] - 2) * (a[2] - 2))
    gbs = RADIATIVE_BYTES_PER_POINT * npts / (ms * 1e-3) / 1e9
    del du, k
    torch.cuda.empty_cache()
    return {"kernel": "k_radiative (all ghost layers, one launch)",
            "ms_per_call": round(ms, 4), "boundary_points": npts,
            "bytes_per_point": RADIATIVE_BYTES_PER_POINT,
            "achieved_gbs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def time_radiative_step(B, torch, g, u_host, prm, steps=10, warmup=2):
    """Whole RK4 steps with the radiative boundary evolved
    (rk4_stage_radiative: the fused interior stage, which also stores the
    right-hand side of the outermost interior layer, then the boundary
    stage update) against the same steps with static ghosts (rk4_stage),
    HIP events on the launch stream."""
    du = torch.from_numpy(u_host).to("cuda")
    a, b, acc, k = (torch.zeros_like(du) for _ in range(4))
    stream = torch.cuda.current_stream()
    res = {}
    for name, step in (("static", lambda: B.rk4_step(
            g, prm, 0.03125, du, a, b, acc, stream)),
                       ("radiative", lambda: B.rk4_step_radiative(
                           g, prm, 0.03125, du, a, b, acc, k,
                           stream=stream))):
        du.copy_(torch.from_numpy(u_host))
        a.copy_(du)
        b.copy_(du)
        acc.copy_(du)
        for _ in range(warmup):
            step()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / steps
    finite = bool(torch.isfinite(du).all().item())
    del du, a, b, acc, k
    torch.cuda.empty_cache()
    return {"kernels": "k_stage_lds (also storing the right-hand side of "
                       "the outermost interior layer), k_radiative_stage "
                       "per stage",
            "ms_per_step_radiative": round(res["radiative"], 4),
            "ms_per_step_static": round(res["static"], 4),
            "overhead": round(res["radiative"] / res["static"] - 1.0, 4),
            "updates_per_s_radiative": round(
                g.npoints / (res["radiative"] * 1e-3), 1),
            "finite": finite}


ADM_BYTES_PER_POINT = 328  # 16 ADM values in, 25 BSSN values out (8 B each)


def time_from_adm(B, torch, g, masses, centres, order, reps=5):
    """bssn_from_adm on the workload's grid and its Brill-Lindquist data in
    ADM form (g_ij = psi^4 delta_ij, K_ij = 0, pre-collapsed lapse), timed
    between HIP events on the launch stream over reps calls."""
    import numpy as np
    X, Y, Z = g.mesh()
    psi = np.ones_like(X)
    for m, c in zip(masses, centres):
        r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
        psi += m / (2.0 * np.maximum(r, 0.5 * min(g.h)))
    adm = torch.zeros(g.off0 + 16 * g.sf, dtype=torch.float64)
    v = g.view(adm.numpy(), 16)
    for s in (0, 3, 5):
        v[s] = psi ** 4
    v[12] = psi ** -2
    del X, Y, Z, psi
    dadm = adm.to("cuda")
    du = torch.empty(g.total, dtype=torch.float64, device="cuda")
    prm = B.Params(fd_order=order)
    stream = torch.cuda.current_stream()
    B.bssn_from_adm(g, prm, dadm, du, stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        B.bssn_from_adm(g, prm, dadm, du, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    npts = 1
    for a in range(3):
        npts *= g.n[a] + 2 * g.ghost
    gbs = ADM_BYTES_PER_POINT * npts / (ms * 1e-3) / 1e9
    del dadm, du
    torch.cuda.empty_cache()
    return {"kernels": "k_adm_point, k_adm_gamma, k_adm_extrap (per layer)",
            "ms_per_call": round(ms, 4), "storage_points": npts,
            "bytes_per_point": ADM_BYTES_PER_POINT,
            "achieved_gbs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def nested_hierarchy(g, nlevel=3):
    """Level 0 the grid g; level L + 1 a patch of the same size at half the
    spacing whose cells split the cells n/4 .. 3n/4 - 1 of level L."""
    from paper_1111_3344_amd import inputs as I
    hier = [(0, g)]
    for L in range(1, nlevel):
        par = hier[-1][1]
        h = tuple(x / 2 for x in par.h)
        o = tuple(par.origin[a] + (par.n[a] // 4 - 0.25) * par.h[a]
                  for a in range(3))
        hier.append((L, I.GridSpec(tuple(par.n), par.ghost, h, o,
                                   I.BC_STATIC)))
    return hier


def split_hierarchy(g, nlevel=3, k=2):
    """nested_hierarchy with every level cut into k x k x k sibling patches
    of n/k points per axis (same lattice, sharing faces): k^3 patches per
    level, whose face ghosts come from their siblings."""
    from paper_1111_3344_amd import inputs as I
    out = []
    for L, gr in nested_hierarchy(g, nlevel):
        m = tuple(x // k for x in gr.n)
        for cz in range(k):
            for cy in range(k):
                for cx in range(k):
                    c = (cx, cy, cz)
                    o = tuple(gr.origin[a] + c[a] * m[a] * gr.h[a]
                              for a in range(3))
                    out.append((L, I.GridSpec(m, gr.ghost, gr.h, o,
                                              I.BC_STATIC)))
    return out


def time_amr_step(B, torch, g, wl, order, steps=3, precision=None,
                  split=1, batched=True):
    """Berger-Oliger stepping (paper_1111_3344_amd.amr) of the workload's
    punctures on three nested levels of its grid (nested_hierarchy, or with
    split > 1 split_hierarchy: split^3 patches per level): one level-0 step
    = 1 + 2 + 4 level steps, a ghost fill per RK4 stage and per level step,
    two restrictions; a level's stages batched over its patches or one
    launch per patch.  One warm-up step, then `steps` steps between device
    synchronisations (host clock)."""
    from paper_1111_3344_amd import amr
    from paper_1111_3344_amd import inputs as I
    hier = nested_hierarchy(g) if split == 1 else split_hierarchy(g, k=split)
    u0 = [B.to_device(I.brill_lindquist(gr, wl[4], wl[5])) for _, gr in hier]
    prm = B.Params(fd_order=order,
                   precision=B.BSSN_FP64 if precision is None else precision)
    drv = amr.BergerOliger(hier, prm, wl[7], u0, batched=batched)
    drv.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        drv.step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    levels = sorted({L for L, _ in hier})
    level_steps = sum(2 ** L for L in levels)
    upd = sum(gr.npoints * 2 ** L for L, gr in hier)
    ok = all(bool(torch.isfinite(x).all()) for x in drv.u)
    del drv, u0
    torch.cuda.empty_cache()
    return {"ms_per_level0_step": round(ms, 3),
            "level_steps_per_level0_step": level_steps,
            "fills_per_level0_step": 5 * (level_steps - 1),
            "updates_per_s": upd / (ms * 1e-3), "finite": ok,
            "hierarchy": "3 nested levels of the workload grid, h, h/2, h/4"
                         + (f", each cut into {split ** 3} patches"
                            if split > 1 else ""),
            "level_stages": ("batched over the level's patches (a level "
                             "of one patch: its rk4_stage)") if batched
                            else "one launch per patch"}


AMR_FILL_BYTES = 232      # 32 B bookkeeping + 25 values written; reads below
AMR_RESTRICT_BYTES = 1832  # op (32 B) + 25 values written + 8 children read


def time_amr_glue(B, torch, g, reps=10):
    """Ghost fill and restriction of a three-level hierarchy on the
    workload's grid: level 0 the grid itself; level 1 and 2 one patch of
    the same size at half and a quarter of the spacing, centred (cells
    n/4 .. 3n/4 of the level below).  Three coarse time levels, target
    time between them.  The state values do not change the work (random
    device data).  Timed between HIP events on the launch stream; the
    pointer tables are built before the timed region."""
    import ctypes
    n = g.n
    hier = nested_hierarchy(g)
    plan = B.AmrPlan(hier)

    def state(gr):
        return torch.randn(gr.total, dtype=torch.float64, device="cuda")

    u = [state(gr) for _, gr in hier]
    old = [[state(gr) for _, gr in hier] for _ in range(2)]
    tabs = [plan._table(x) for x in (u, old[0], old[1])]
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    L = B.lib()
    ts = (ctypes.c_double * 3)(0.0, 1.0, 2.0)
    src = (ctypes.c_void_p * 3)(tabs[1].value, tabs[2].value, tabs[0].value)

    def fill(level):
        B._check(L.bssn_amr_fill_ghosts(plan.h, level, tabs[0], 3, src, ts,
                                        1.25, sp))

    def restrict(level):
        B._check(L.bssn_amr_restrict(plan.h, level, tabs[0], tabs[0], sp))

    res = {}
    for name, fn, level in (("fill_level1", fill, 1), ("fill_level2", fill, 2),
                            ("restrict_level1", restrict, 1),
                            ("restrict_level2", restrict, 2)):
        fn(level)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn(level)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        nfill, ncopy, nrestr = plan.counts(level)
        if name.startswith("fill"):
            nops = nfill
            # each coarse value serves about 8 fine points (3 time levels)
            bpo = AMR_FILL_BYTES + 3 * 200 / 8
        else:
            nops = nrestr
            bpo = AMR_RESTRICT_BYTES
        gbs = nops * bpo / (ms * 1e-3) / 1e9
        res[name] = {"ms_per_call": round(ms, 4), "points": int(nops),
                     "bytes_per_point": bpo, "achieved_gbs": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK_GBS, 4)}
    plan.destroy()
    del u, old
    torch.cuda.empty_cache()
    res["hierarchy"] = (f"3 levels of {n[0]}x{n[1]}x{n[2]} + {g.ghost} "
                        f"ghosts, spacings h, h/2, h/4, nested centred")
    return res


def time_multipole(B, torch, g, reps=10):
    """bssn_multipole of a complex field (the real and imaginary parts two
    slots of a state on the workload's grid) on the sphere r = 0.75 of the
    half-width around the grid centre, spin -2, l <= 8, 64 x 128 points."""
    import ctypes
    u = torch.randn(g.total, dtype=torch.float64, device="cuda")
    centre = [g.origin[a] + (g.n[a] - 1) * g.h[a] / 2 for a in range(3)]
    radius = 0.75 * (g.n[0] - 1) * g.h[0] / 2
    nt, nph, lmax = 64, 128, 8
    chunks = min(64, (nt * nph + 255) // 256)
    work = torch.empty(2 * nt * (nph + 1) + 2 * (lmax + 1) ** 2 * chunks,
                       dtype=torch.float64, device="cuda")
    coeffs = torch.empty(2 * (lmax + 1) ** 2, dtype=torch.float64,
                         device="cuda")
    c = (ctypes.c_double * 3)(*centre)
    rp = ctypes.c_void_p(B.ptr(g, u).value + 8 * 17 * g.sf)
    ip = ctypes.c_void_p(B.ptr(g, u).value + 8 * 7 * g.sf)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    L = B.lib()

    def call():
        B._check(L.bssn_multipole(ctypes.byref(B.c_grid(g)), rp, ip, c,
                                  radius, -2, lmax, nt, nph,
                                  ctypes.c_void_p(work.data_ptr()),
                                  ctypes.c_void_p(coeffs.data_ptr()), sp))
    call()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        call()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del u, work, coeffs
    return {"kernels": "k_gl_nodes, k_sphere_interp, k_multipole, "
                       "k_multipole_sum",
            "ms_per_call": round(ms, 4), "sphere_points": nt * nph,
            "lmax": lmax, "spin": -2, "radius": radius}


PSI4_BYTES = 128  # phi, gt_ij, K, At_ij in (14 slots), Re and Im out


def time_psi4(B, torch, g, u_host, order, reps=10):
    """bssn_psi4 over the whole grid (tetrad centred a little off the
    origin), HIP events on the launch stream; algorithmic bytes 128 per
    interior point."""
    du = torch.from_numpy(u_host).to("cuda")
    out = torch.zeros(g.off0 + 2 * g.sf, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    centre = (0.013, -0.021, 0.007)
    B.bssn_psi4(g, order, du, out, centre, stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        B.bssn_psi4(g, order, du, out, centre, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    finite = bool(torch.isfinite(out).all().item())
    del du, out
    torch.cuda.empty_cache()
    gbs = g.npoints * PSI4_BYTES / (ms * 1e-3) / 1e9
    return {"kernel": f"k_psi4<{order}>", "ms_per_call": round(ms, 4),
            "points": g.npoints, "bytes_per_point": PSI4_BYTES,
            "achieved_gbs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "finite": finite}


def cpu_model():
    """The host CPU's model name (/proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(name, target_s=15.0, width=128):
    """The oracle on the host cores over a bounded sample of the workload:
    a width x width x nz box of the same grid around its centre (same data,
    static ghosts taken from the full grid's initial data), whole RK4 steps,
    with as many threads as this process may run on.  The oracle's loops are
    parallel over z planes, so nz is a multiple of the thread count: a probe
    of one plane per thread sets it so that the sample takes about target_s.
    One thread on a one-plane box gives the single-core rate."""
    import numpy as np
    from oracle import oracle as O
    from paper_1111_3344_amd import inputs as I
    n, lo, hi, gh, masses, centres, order, dt, desc = WORKLOADS[name]
    h = (hi - lo) / n
    w = min(width, n)
    prm = O.params(fd_order=order)
    cores = len(os.sched_getaffinity(0))
    O.set_num_threads(cores)
    threads = O.num_threads()

    def box(nz):
        x0, z0 = n // 2 - w // 2, n // 2 - nz // 2
        g = I.GridSpec((w, w, nz), gh, (h, h, h),
                       (lo + (0.5 + x0) * h, lo + (0.5 + x0) * h,
                        lo + (0.5 + z0) * h), I.BC_STATIC)
        u = (I.brill_lindquist(g, masses, centres) if masses else
             I.minkowski_noise(g))
        return g, u

    def rate(g, u, steps=1):
        t0 = time.perf_counter()
        for _ in range(steps):
            u = O.rk4_step(g, prm, dt, u)
        t = time.perf_counter() - t0
        return g.npoints * steps / t, t

    g, u = box(threads)
    r0, _ = rate(g, u)
    nz = threads * int(max(1, round(target_s * r0 / (w * w * threads))))
    nz = min(nz, n)
    g, u = box(nz)
    r, t = rate(g, u)
    O.set_num_threads(1)
    g1, u1 = box(1)
    r1, t1 = rate(g1, u1)
    O.set_num_threads(cores)
    return {"value": r, "unit": "grid-point updates/s",
            "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "one_thread_value": r1,
            "sample": f"1 RK4 step of the FP64 oracle on a {w}x{w}x{nz} box "
                      f"at the centre of {name} ({g.npoints} point updates, "
                      f"{t:.1f} s, {threads} threads); one thread: 1 step "
                      f"on a {w}x{w}x1 box ({t1:.1f} s)"}


# ---- rocprofv3 summaries ------------------------------------------------------
KERNEL_SOURCES = ("bssn_internal.h", "bssn_point.h", "bssn_stage.h",
                  "bssn_lds.h", "bssn_rhs_o4.hip", "bssn_rhs_o8.hip")
CALIB_BYTES = 1 << 30


def strip_comments(src):
    """C/C++ source without comments and with whitespace runs collapsed, so
    that only code changes change the hash (no string in these sources
    contains a comment marker)."""
    import re
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_source_hash(sources=None):
    """Hash of the kernel sources' code (comments and layout ignored)."""
    import hashlib
    hsh = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1111_3344_amd", "csrc")
    for f in KERNEL_SOURCES:
        if sources is not None:
            text = sources[f]
        else:
            with open(os.path.join(d, f)) as fh:
                text = fh.read()
        hsh.update(strip_comments(text).encode())
    return hsh.hexdigest()[:16]


def calibrate_copy(torch):
    """Three plain device-to-device copies of CALIB_BYTES, last in the run."""
    a = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


def _csv_rows(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def summarize_profile(dirs, order=4):
    """Text summary of rocprofv3 CSV output directories: per-kernel dispatch
    durations (kernel trace) and per-dispatch counter values (pmc runs).
    Lines starting with '#' are the summary; the 'key: value' lines at the
    end are the figures bench.py reads back for the FP64 stage kernel of the
    given order (HBM bytes per launch scaled by the copy calibration, VALU
    FLOPs per launch) and, prefixed mixed_, for the two launches of a mixed
    stage, stamped with the hash of the kernel sources."""
    import glob
    import collections
    import re
    out = []
    # the production instantiations (the second template argument, false,
    # is the radiative-boundary variant's switch)
    tail = r"\s*(,\s*false\s*)?>\("
    kernels = (("", re.compile(r"k_stage_lds<\s*%d" % order + tail)),
               ("mixed_f32_", re.compile(r"k_stage_lds_f32<\s*%d" % order +
                                         tail)),
               ("mixed_f64pass_", re.compile(
                   r"k_stage_lds_f64tiles<\s*%d" % order + tail)))

    def tag(name):
        for t, rx in kernels:
            if rx.search(name):
                return t
        return None
    kv = {}
    for d in dirs:
        for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"),
                                  recursive=True)):
            dur = collections.defaultdict(list)
            for r in _csv_rows(f):
                dur[r["Kernel_Name"]].append(
                    int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
            out.append(f"# kernel trace: {os.path.relpath(f, d)}")
            out.append("#  calls    avg_us    min_us    max_us  total_ms  "
                       "kernel")
            for k, v in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
                out.append(f"# {len(v):6d} {sum(v) / len(v) / 1e3:9.1f} "
                           f"{min(v) / 1e3:9.1f} {max(v) / 1e3:9.1f} "
                           f"{sum(v) / 1e6:9.2f}  {k[:110]}")
                if tag(k) is not None:
                    kv[tag(k) + "avg_launch_us"] = \
                        f"{sum(v) / len(v) / 1e3:.2f}"
        for f in sorted(glob.glob(os.path.join(d, "**",
                                               "*counter_collection.csv"),
                                  recursive=True)):
            per = collections.defaultdict(dict)
            names = {}
            for r in _csv_rows(f):
                did = int(r["Dispatch_Id"])
                per[did][r["Counter_Name"]] = (
                    per[did].get(r["Counter_Name"], 0.0) +
                    float(r["Counter_Value"]))
                names[did] = r["Kernel_Name"]
            out.append(f"# counters: {os.path.relpath(f, d)}")
            agg = collections.defaultdict(lambda: collections.defaultdict(list))
            for did in sorted(per):
                for c, v in per[did].items():
                    agg[names[did]][c].append(v)
            for k, cs in agg.items():
                for c, v in cs.items():
                    out.append(f"#   {c:26s} dispatches {len(v):4d} avg "
                               f"{sum(v) / len(v):14.6g}  {k[:90]}")
                    if tag(k) is not None:
                        kv[f"{tag(k)}{c}_per_launch"] = sum(v) / len(v)
            copies = [did for did in sorted(per)
                      if "copyBuffer" in names[did]][-3:]
            for c in sorted({c for did in copies for c in per[did]}):
                v = [per[did][c] for did in copies]
                out.append(f"#   calibration: {c} over {len(v)} plain "
                           f"copies of {CALIB_BYTES} bytes, avg "
                           f"{sum(v) / len(v):.6g}")
                kv[f"copy_{c}"] = sum(v) / len(v)
    res = [f"source_sha256: {kernel_source_hash()}"]
    for t, _ in kernels:
        if t + "avg_launch_us" in kv:
            res.append(f"{t}avg_launch_us: {kv[t + 'avg_launch_us']}")
    if all(k in kv for k in ("copy_FETCH_SIZE", "copy_WRITE_SIZE")):
        res += [f"copy_bytes: {CALIB_BYTES}",
                f"copy_fetch_kib: {kv['copy_FETCH_SIZE']:.6g}",
                f"copy_write_kib: {kv['copy_WRITE_SIZE']:.6g}"]
        for t, _ in kernels:
            if all(f"{t}{c}_per_launch" in kv
                   for c in ("FETCH_SIZE", "WRITE_SIZE")):
                res += [f"{t}fetch_kib_per_launch: "
                        f"{kv[t + 'FETCH_SIZE_per_launch']:.6g}",
                        f"{t}write_kib_per_launch: "
                        f"{kv[t + 'WRITE_SIZE_per_launch']:.6g}"]
    for t, _ in kernels:
        for prec in ("F64", "F32"):
            parts = [f"{t}SQ_INSTS_VALU_{o}_{prec}_per_launch"
                     for o in ("ADD", "MUL", "FMA", "TRANS")]
            if all(p in kv for p in parts):
                a, m, fma, tr = (kv[p] for p in parts)
                res.append(f"{t}valu_flops_{prec.lower()}_per_launch: "
                           f"{64 * (a + m + tr + 2 * fma):.6g}")
    return "\n".join(out + res)


def profile_figures(workload, kernel_tag):
    """The key: value figures of the committed counter summary for this
    kernel and workload, or (None, reason) when there is none or the kernel
    sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles",
                        f"traffic_{kernel_tag}_{workload}.txt")
    if not os.path.exists(path):
        return None, "no counter summary for this workload"
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash():
        return None, "kernel sources changed since the counters were taken"
    return kv, os.path.relpath(path, ROOT)


def traffic_bytes(kv, prefix=""):
    """Measured HBM bytes per launch of the kernel the prefix names: each
    counter scaled by what it reads for a plain copy of known size."""
    f = float(kv[prefix + "fetch_kib_per_launch"]) * 1024.0
    w = float(kv[prefix + "write_kib_per_launch"]) * 1024.0
    fc = float(kv["copy_fetch_kib"]) * 1024.0
    wc = float(kv["copy_write_kib"]) * 1024.0
    cb = float(kv["copy_bytes"])
    return f * cb / fc + w * cb / wc


def batched(B, torch, steps, warmup, npatch=256):
    """256 uneven static patches (interiors U{24..96} per axis, h = 0.125,
    one Brill-Lindquist puncture each): a batch plan advanced with
    batch_patches (one graph replay per RK4 step) against one launch per
    patch and stage, FP64 and mixed.  The plan is autotuned (tile per size
    class and launch mode), and a second plan forced to the persistent
    work-list mode is timed too."""
    from paper_1111_3344_amd import inputs as I
    specs = I.patches(npatch)
    grids = [g for g, _, _ in specs]
    u = []
    for g, m, c in specs:  # host copies one at a time
        u.append(torch.from_numpy(I.brill_lindquist(g, (m,), (c,))).to("cuda"))
    a = [t.clone() for t in u]
    b = [t.clone() for t in u]
    acc = [torch.zeros_like(t) for t in u]
    N = sum(g.npoints for g in grids)
    stream = torch.cuda.current_stream()
    out = {"interior_points": N, "npatch": npatch}
    for label, prec in (("f64", B.BSSN_FP64), ("mixed", B.BSSN_MIXED)):
        plan = B.batch_patches_plan(grids, B.Params(precision=prec), u, a, b,
                                    acc, 0.03125, autotune=True)
        r = {"classes": [list(c) for c in B.batch_patches_describe(plan)],
             "launch_mode": ("per-patch graph" if
                             B.batch_patches_launch_mode(plan) else
                             "persistent work lists")}
        forced = B.batch_patches_plan(grids, B.Params(precision=prec), u, a,
                                      b, acc, 0.03125,
                                      autotune=B.BSSN_BATCH_TILE(0))
        for mode, fn, pl in (("batched", B.batch_patches, plan),
                             ("batched_persistent", B.batch_patches, forced),
                             ("per_patch", B.batch_patches_unbatched, plan)):
            fn(pl, warmup, stream)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record(stream)
            fn(pl, steps, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            r[mode] = {"value": N * steps / wall,
                       "ms_per_step": 1e3 * wall / steps,
                       "gpu_ms_per_step": e0.elapsed_time(e1) / steps,
                       "hbm_frac": round(3200.0 * N * steps / wall / 1e9 /
                                         HBM_PEAK_GBS, 4)}
        plan.destroy()
        forced.destroy()
        out[label] = r
    return out


ACCURACY_STEPS = {"noise32": 1, "bl1-128": 100, "bl2-256": 200,
                  "bl2-384-o8": 50}


def accuracy(B, torch, name, steps=None, r_exc=1.0):
    """FP64 and mixed-precision runs of a workload for its step count: the
    mixed run's field error against the FP64 run (per slot, normwise: max
    and L2 of |mixed - fp64| over max |fp64| of that slot; the FP64 path
    matches the oracle to 1e-12 per step) and both runs' constraint norms
    (points closer than r_exc to a puncture left out)."""
    g, u, order, dt, desc = build_state(name)
    steps = steps or ACCURACY_STEPS[name]
    centres = WORKLOADS[name][5] or ()
    res = {}
    ref = None
    for label, prec in (("f64", B.BSSN_FP64), ("mixed", B.BSSN_MIXED)):
        prm = B.Params(fd_order=order, precision=prec)
        du = torch.from_numpy(u).to("cuda")
        a, b, acc = du.clone(), du.clone(), torch.zeros_like(du)
        t0 = time.perf_counter()
        for _ in range(steps):
            B.rk4_step(g, prm, dt, du, a, b, acc)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        del a, b, acc
        norms = torch.zeros(8, dtype=torch.float64, device="cuda")
        B.bssn_constraints(g, B.Params(fd_order=order), du, norms,
                           centres=centres, r_exc=r_exc if centres else 0.0)
        n = norms.cpu().numpy()
        r = {"H_rms": n[0], "H_max": n[1], "M_rms": n[2], "M_max": n[3],
             "G_rms": n[4], "points": int(n[6]), "nonfinite": int(n[7]),
             "seconds": round(wall, 3)}
        if prec == B.BSSN_MIXED:
            n64, nt = B.bssn_mixed_tile_count(g, prm, du)
            r["fp64_tiles"] = f"{n64}/{nt} (final state)"
        if ref is None:
            ref = du
        else:
            mx, l2 = [], []
            for sl in range(25):
                x = g.interior(ref)[sl]
                y = g.interior(du)[sl]
                D = float(x.abs().max())
                D = D if D > 0 else 1.0
                d = (y - x).abs()
                mx.append(float(d.max()) / D)
                l2.append(float(d.pow(2).mean().sqrt()) / D)
            r["field_err_vs_f64_max"] = max(mx)
            r["field_err_vs_f64_l2"] = max(l2)
            r["worst_slot"] = mx.index(max(mx))
            r["H_rms_ratio"] = r["H_rms"] / res["f64"]["H_rms"]
            r["M_rms_ratio"] = r["M_rms"] / res["f64"]["M_rms"]
            del du
        res[label] = r
    return {"accuracy": name, "workload": desc, "steps": steps, "dt": dt,
            "r_exc": r_exc if centres else None, **res}


def run_grid(B, torch, name, steps, warmup, mixed=True):
    """FP64 (and mixed-precision) RK4 steps of a single-grid workload:
    wall-clock updates/s and the HIP-event duration of every stage kernel."""
    g, u, order, dt, desc = build_state(name)
    N = g.npoints
    res = {}
    for label, prec in (("f64", B.BSSN_FP64), ("mixed", B.BSSN_MIXED)):
        if label == "mixed" and not mixed:
            continue
        prm = B.Params(fd_order=order, precision=prec)
        wall, per_stage = time_gpu(B, torch, g, u, prm, dt, steps, warmup)
        kern_ms = sum(per_stage)
        ach = sum(b * N for b in STAGE_BYTES) / (kern_ms * 1e-3) / 1e9
        res[label] = {"value": N * steps / wall,
                      "ms_per_step": 1e3 * wall / steps,
                      "stage_kernel_ms": [round(x, 4) for x in per_stage],
                      "achieved_gbs": ach}
    return g, u, order, dt, desc, res


def grid_summary(res):
    """Compact FP64 / mixed figures of run_grid for a secondary line."""
    out = {}
    for label, r in res.items():
        out[label] = {"value": r["value"],
                      "ms_per_step": round(r["ms_per_step"], 3),
                      "hbm_frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                      "stage_kernel_ms": r["stage_kernel_ms"]}
    return out


COPY_BYTES = 4 << 30


def copy_bandwidth(torch, nbytes=COPY_BYTES, reps=5):
    """HBM bandwidth of a plain device-to-device copy of nbytes (read +
    write counted), best of reps, on the same GPU in the same run."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def constraint_norms_after(B, torch, name, steps, r_exc=1.0):
    """Hamiltonian and momentum constraint norms of a workload after
    `steps` FP64 RK4 steps from its initial data: RMS over every interior
    point, and over the points farther than r_exc from each puncture."""
    g, u, order, dt, desc = build_state(name)
    centres = WORKLOADS[name][5]
    prm = B.Params(fd_order=order)
    du = torch.from_numpy(u).to("cuda")
    a, b, acc = du.clone(), du.clone(), torch.zeros_like(du)
    out = {"steps": steps, "t": steps * dt, "precision": "f64"}
    for k in range(steps + 1):
        if k in (0, steps):
            for key, c, r in (("all", (), 0.0), ("masked", centres, r_exc)):
                n = torch.zeros(8, dtype=torch.float64, device="cuda")
                B.bssn_constraints(g, prm, du, n, centres=c, r_exc=r)
                v = n.cpu().numpy()
                out[f"{key}_t{'0' if k == 0 else 'end'}"] = {
                    "H_rms": float(v[0]), "H_max": float(v[1]),
                    "M_rms": float(v[2]), "points": int(v[6]),
                    "nonfinite": int(v[7])}
        if k < steps:
            B.rk4_step(g, prm, dt, du, a, b, acc)
    torch.cuda.synchronize()
    out["r_exc"] = r_exc
    del du, a, b, acc
    torch.cuda.empty_cache()
    return out


def psi4_o8_state(I, wl):
    """The workload's grid and data with the 5 ghost layers of order 8."""
    n, lo, hi, gh, masses, centres = wl[:6]
    g = I.cell_centred(n, lo, hi, 5)
    return g, I.brill_lindquist(g, masses, centres)


def extras(B, torch, name, order):
    """The steps around the path, timed on a workload's grid: radiative
    boundary, ADM->BSSN conversion, refinement glue, multipole and
    Berger-Oliger stepping."""
    from paper_1111_3344_amd import inputs as I
    wl = WORKLOADS[name]
    g, u, order, dt, desc = build_state(name)
    out = {"grid": name,
           "radiative_bc": time_radiative(B, torch, g, u,
                                          B.Params(fd_order=order)),
           "radiative_step": time_radiative_step(B, torch, g, u,
                                                 B.Params(fd_order=order)),
           "adm_to_bssn": time_from_adm(B, torch, g, wl[4], wl[5], order),
           "amr_glue": time_amr_glue(B, torch, g),
           "multipole": time_multipole(B, torch, g),
           "psi4": time_psi4(B, torch, g, u, order),
           "psi4_o8": time_psi4(B, torch, *psi4_o8_state(I, wl), 8),
           "amr_berger_oliger": time_amr_step(B, torch, g, wl, order),
           "amr_berger_oliger_mixed": time_amr_step(
               B, torch, g, wl, order, precision=B.BSSN_MIXED),
           "amr_berger_oliger_8patches": time_amr_step(
               B, torch, g, wl, order, split=2),
           "amr_berger_oliger_8patches_per_patch": time_amr_step(
               B, torch, g, wl, order, split=2, batched=False)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bl2-384-o8",
                    choices=list(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline workload (no secondary "
                         "workloads, extras or copy measurement)")
    ap.add_argument("--path", default="auto", choices=["auto", "direct"],
                    help="kernel: LDS-pipelined (auto) or direct-load")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with three 1 GiB device copies (counter "
                         "calibration under rocprofv3 --pmc)")
    ap.add_argument("--accuracy", action="store_true",
                    help="FP64 vs mixed runs of the workload for its step "
                         "count: field errors and constraint norms")
    ap.add_argument("--psi4-only", action="store_true",
                    help="only time bssn_psi4 (orders 4 and 8) on the "
                         "workload's grid")
    ap.add_argument("--amr-glue-only", action="store_true",
                    help="only the refinement-glue timing on the workload's "
                         "grid (JSON line)")
    ap.add_argument("--summarize-profile", nargs="+", metavar="DIR",
                    help="print a text summary of rocprofv3 CSV output "
                         "directories and exit")
    args = ap.parse_args()
    if args.summarize_profile:
        print(summarize_profile(args.summarize_profile,
                                WORKLOADS[args.workload][6]))
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for "
              f"{args.gpus}); the multi-GPU design is documented but not "
              "built", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1111_3344_amd import bssn as B

    B.bssn_set_path(B.BSSN_PATH_DIRECT if args.path == "direct"
                    else B.BSSN_PATH_AUTO)
    if args.workload == "patches256":
        r = batched(B, torch, args.steps, args.warmup)
        print(json.dumps({"workload": WORKLOADS["patches256"][8],
                          "steps": args.steps, "warmup": args.warmup, **r}),
              flush=True)
        return
    if args.accuracy:
        print(json.dumps(accuracy(B, torch, args.workload)), flush=True)
        return
    if args.psi4_only:
        from paper_1111_3344_amd import inputs as I
        wl = WORKLOADS[args.workload]
        g, u, order, dt, desc = build_state(args.workload)
        print(json.dumps({"workload": args.workload,
                          "psi4": time_psi4(B, torch, g, u, order),
                          "psi4_o8": time_psi4(B, torch,
                                               *psi4_o8_state(I, wl), 8)}),
              flush=True)
        if args.calibrate_copy:
            calibrate_copy(torch)
        return
    if args.amr_glue_only:
        from paper_1111_3344_amd import inputs as I
        wl = WORKLOADS[args.workload]
        gg = I.cell_centred(wl[0], wl[1], wl[2], wl[3])
        print(json.dumps({"workload": args.workload,
                          "amr_glue": time_amr_glue(B, torch, gg)}),
              flush=True)
        return
    g, u, order, dt, desc, res = run_grid(B, torch, args.workload,
                                          args.steps, args.warmup,
                                          mixed=not args.no_mixed)
    del u
    N = g.npoints
    if args.calibrate_copy:
        calibrate_copy(torch)
    f = res["f64"]
    lds = args.path == "auto"
    kernel = f"k_stage_lds<{order}>" if lds else f"k_stage<{order},...>"
    kv, tsrc = (profile_figures(args.workload, f"k_stage_lds_o{order}")
                if lds else (None, "no counter summary for this kernel"))
    traffic = traffic_bytes(kv) if kv and "fetch_kib_per_launch" in kv \
        else None
    avg_s = sum(f["stage_kernel_ms"]) / 4 * 1e-3
    out = {
        "metric": "BSSN RHS+RK4 grid-point updates/s, FP64 vs mixed, % of "
                  "HBM roofline",
        "value": f["value"],
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "name": args.workload,
                   "interior_points": N, "fd_order": order, "dt": dt},
        "roofline": {"bound": "hbm", "achieved": round(f["achieved_gbs"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(f["achieved_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": (None if traffic is None else
                                 round(traffic)),
                     "traffic_unit": "HBM bytes per stage launch (mean of "
                                     "the 4 stages)",
                     "traffic_source": tsrc,
                     "algorithmic_bytes_per_launch":
                         sum(b * N for b in STAGE_BYTES) / 4,
                     "kernel": kernel + " (fused RHS + RK4 stage)",
                     "avg_launch_ms": round(sum(f["stage_kernel_ms"]) / 4, 4),
                     "stage_kernel_ms": f["stage_kernel_ms"]},
    }
    if kv and "valu_flops_f64_per_launch" in kv:
        fl = float(kv["valu_flops_f64_per_launch"])
        out["valu"] = {"flops_f64_per_launch": fl,
                       "achieved": round(fl / avg_s / 1e12, 2),
                       "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(fl / avg_s / 1e12 / FP64_PEAK_TFLOPS, 4),
                       "source": tsrc}
    if "mixed" in res:
        m = res["mixed"]
        out["mixed"] = {"value": m["value"], "ms_per_step": m["ms_per_step"],
                        "dtype": "f32 stencils/algebra, f64 state and RK4",
                        "roofline_frac": round(m["achieved_gbs"] /
                                               HBM_PEAK_GBS, 4),
                        "achieved_gbs": round(m["achieved_gbs"], 1),
                        "stage_kernel_ms": m["stage_kernel_ms"],
                        "speedup_vs_f64": round(m["value"] / f["value"], 4)}
        if lds:
            out["mixed"]["kernels"] = (
                f"k_stage_lds_f32<{order}> (FP32 tiles) then "
                f"k_stage_lds_f64tiles<{order}> (FP64 tiles), per stage")
            if kv and "mixed_f32_fetch_kib_per_launch" in kv:
                t32 = traffic_bytes(kv, "mixed_f32_")
                t64 = (traffic_bytes(kv, "mixed_f64pass_") if
                       "mixed_f64pass_fetch_kib_per_launch" in kv else 0.0)
                out["mixed"]["traffic"] = round(t32 + t64)
                out["mixed"]["traffic_unit"] = ("HBM bytes per stage (both "
                                                "launches, mean of the 4 "
                                                "stages)")
                out["mixed"]["traffic_source"] = tsrc
            for t in ("mixed_f32_", "mixed_f64pass_"):
                if kv and t + "avg_launch_us" in kv:
                    out["mixed"][t[6:] + "profiled_avg_launch_us"] = float(
                        kv[t + "avg_launch_us"])
    if not args.no_extra:
        cp = copy_bandwidth(torch)
        out["copy"] = {"gbs": round(cp, 1), "bytes": COPY_BYTES,
                       "what": "device-to-device copy (read + write), best "
                               "of 5, same GPU and run"}
        out["roofline"]["frac_of_copy"] = round(f["achieved_gbs"] / cp, 4)
        if "mixed" in out:
            out["mixed"]["frac_of_copy"] = round(
                res["mixed"]["achieved_gbs"] / cp, 4)
        wk = {}
        for name in ("bl2-256", "bl1-128"):
            if name == args.workload:
                continue
            *_, r = run_grid(B, torch, name, args.steps, args.warmup,
                             mixed=not args.no_mixed)
            wk[name] = {"workload": WORKLOADS[name][8], **grid_summary(r)}
        wk.setdefault("bl1-128", {})["constraints_100_steps"] = \
            constraint_norms_after(B, torch, "bl1-128", 100)
        wk["patches256"] = {"workload": WORKLOADS["patches256"][8],
                            **batched(B, torch, args.steps, args.warmup)}
        out["workloads"] = wk
        out["extras"] = extras(B, torch, "bl1-128", 4)
        # mixed precision against FP64 over each workload's full run:
        # field error and constraint norms (the mixed form's bound)
        out["accuracy"] = {name: accuracy(B, torch, name)
                           for name in ("bl2-384-o8", "bl2-256")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
