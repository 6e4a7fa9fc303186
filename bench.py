"""Benchmark of the RK3 immersed-boundary step on one MI355X.

Workload (default): the FP64 sinusoidal-wall channel, 512x257x256 cells-faces
(512 x 256 x 256 = 33,554,432 cells, larger than the 256 MB Infinity Cache, so an HBM
roofline case), constant flow rate at Re_bulk = 2800, dt = 0.003, seeded synthetic
inputs (no dataset).  One "step" is one full RK3
time step = 3 substeps of the whole hot path (momentum + immersed-boundary
update + flow-rate control + FFT/tridiagonal projection + correction).

Prints ONE JSON line with the throughput in cell-updates per second per RK
substep, the roofline figures of the dominant kernel (timed live with HIP
events on the library's stream during the timed region), the FP64 CPU oracle
timed on a bounded sample, and the other measured forms.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per RK substep + % HBM peak; FP64 vs FP32-storage vs batched"
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="wavy_large", help="wavy_large | wavy | wavy_open | ellipsoids | poiseuille")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--projection", default="full", choices=["full", "masked"],
                    help="pressure projection of the main workload (masked: FP64, conjugate gradients)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the extra forms (FP32, large grid, IBM off)")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup + steps without extra forms or baseline (for rocprofv3)")
    ap.add_argument("--tuning", default="",
                    help="fixed tuning knobs instead of the autotuner, e.g. momentum_planes=12,fftz_width=8")
    ap.add_argument("--only-form", default="", choices=["", "ensemble", "masked", "moving", "shards"],
                    help="run only this extra form (its own step counts, or --steps for the ensemble), print "
                         "its JSON and exit (for rocprofv3 traces of the form)")
    ap.add_argument("--stream-table", action="store_true",
                    help="print the HBM throughput of the library's stream kernels for several numbers "
                         "of read and write streams (arrays of one 512x257x256 field) and exit")
    ap.add_argument("--copy-calibration-mb", type=float, default=0.0,
                    help="also run the library's streaming copy of this many MiB three times (PMC counter "
                         "calibration)")
    return ap.parse_args()


# --------------------------------------------------------------------------------------
# Algorithmic HBM bytes per launch of each kernel (values that must move at least once).
#   C = cells, M = spectral points (nx/2+1)*nz*(ny-1), s = bytes per stored value,
#   n_ibm = immersed-boundary points (all components), n_u = those of u.
# --------------------------------------------------------------------------------------
def algorithmic_bytes(kernel, C, M, s, n_ibm, n_u):
    if kernel == "momentum":
        # the previous substep's projection folded in: reads u*', v*', w*', p', phi, tag,
        # H_prev (stages 2, 3); writes u*, v*, w*, p, H (stages 1, 2): avg 13 fields + tag;
        # (B, 1/A) of every immersed-boundary point
        return C * (13 * s + 1) + n_ibm * 16
    if kernel == "div_fftx":
        # reads u*, v*, w*, tag; writes the x-spectrum
        return C * (3 * s + 1) + M * 2 * s
    if kernel in ("fftz_fwd", "fftz_inv", "tri"):
        return M * 4 * s
    if kernel == "ifftx":
        return M * 2 * s + C * s
    if kernel == "correct":
        # materialising the state on request (not part of a step)
        return C * (9 * s + 1)
    if kernel == "cfr_pi":
        # index, 1/A and u* read-modify-write of each immersed-boundary u face (the flow-rate
        # partials are a few kB)
        return n_u * (4 + 8 + 2 * s)
    raise KeyError(kernel)


def step_bytes(C, M, s, n_ibm, n_u):
    per_sub = sum(algorithmic_bytes(k, C, M, s, n_ibm, n_u) for k in
                  ("momentum", "cfr_pi", "div_fftx", "fftz_fwd", "tri", "fftz_inv", "ifftx"))
    return 3 * per_sub


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("kernels_step.hip", "fft_lds.h", "ibm_internal.h"):
        with open(os.path.join(ROOT, "paper_2506_14328_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload, precision):
    """HBM traffic per launch from the committed rocprofv3 PMC summary, if it was taken on
    the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{precision}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_digest") != kernel_source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def build_inputs(name):
    import numpy as np
    import ibm_inputs as I
    c = I.make_case(name)
    sdf = I.make_sdf(c)
    u, v, w = I.make_initial(c, sdf)
    return c, sdf, (u, v, w, np.zeros_like(u))


def make_grid(c, sdf, st, precision, ibm=True):
    import torch
    from paper_2506_14328_amd import IbmGrid
    dev = torch.device("cuda", 0)
    dt = torch.float64 if precision == "fp64" else torch.float32
    g = IbmGrid.from_case(c, precision=precision, ibm=ibm)
    g.set_geometry(*[torch.as_tensor(a).to(dev) for a in sdf])
    g.set_state(*[torch.as_tensor(a).to(dev, dt) for a in st])
    return g


def timed_run(g, steps, warmup, profile_kernel=None):
    """Warmup, then exactly `steps` steps between two device synchronisations.
    With profile_kernel, HIP events bracket every launch of that kernel."""
    import torch
    g.step(warmup)
    if profile_kernel:
        g.profile([profile_kernel])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = g.profile_read() if profile_kernel else {}
    g.profile(False)
    return el, prof


def dominant_kernel(g, nsteps=3):
    """The kernel with the largest total time, each kernel timed in a pass of its own."""
    names = [n for n in g.kernel_names() if n not in ("diag", "stats", "geom", "wall_shear", "pcg")]
    tot = {}
    for n in names:
        g.profile([n])
        g.step(nsteps)
        prof = g.profile_read()
        if n in prof:
            tot[n] = prof[n][0]
    g.profile(False)
    s = sum(tot.values())
    k = max(tot, key=lambda n: tot[n])
    return k, {n: round(100.0 * v / s, 1) for n, v in tot.items()}


def measure(name, precision, steps, warmup, ibm=True, inputs=None, tuning=None, keep_state=False):
    """tuning: None runs the autotuner; a dict sets those knobs."""
    c, sdf, st = inputs if inputs is not None else build_inputs(name)
    g = make_grid(c, sdf, st, precision, ibm)
    stats0 = g.stats()
    if tuning is None:
        # trials of a few milliseconds each, so that timing noise does not decide
        tuned = g.autotune(max(2, min(10, round(1.5e7 / (c.nx * (c.ny - 1) * c.nz)))))
    else:
        g.tune(**tuning)
        tuned = g.tuning()
    kern, shares = dominant_kernel(g)
    g.set_state(*[__import__("torch").as_tensor(a).to("cuda", g.dtype) for a in st])
    el, prof = timed_run(g, steps, warmup, kern)
    C = c.nx * (c.ny - 1) * c.nz
    M = (c.nx // 2 + 1) * c.nz * (c.ny - 1)
    s = 8 if precision == "fp64" else 4
    n_ibm = sum(stats0["n_ibm"])
    ms, cnt = prof[kern]
    avg_s = ms / cnt * 1e-3
    abytes = algorithmic_bytes(kern, C, M, s, n_ibm, stats0["n_ibm"][0])
    achieved = abytes / avg_s / 1e9
    stats = g.stats()
    state = [t.double().cpu().numpy() for t in g.get_state()] if keep_state else None
    g.close()
    return dict(case=c, cells=C, el=el, value=C * 3 * steps / el, ms_per_step=el / steps * 1e3,
                kernel=kern, kernel_avg_us=avg_s * 1e6, kernel_launches=cnt, kernel_bytes=abytes,
                achieved_gbs=achieved, shares=shares, stats=stats, tuning=tuned, state=state,
                step_gbs=step_bytes(C, M, s, n_ibm, stats0["n_ibm"][0]) * steps / el / 1e9,
                ibm_fraction=n_ibm / (3.0 * C))


def precision_errors(a64, a32):
    """Error of the FP32-storage state against the FP64 one.

    "velocity" is the relative velocity error the 1e-5 target refers to: the largest
    difference of any velocity component divided by the largest speed component of the
    FP64 field (max_rel), and the 2-norm of the difference of the whole velocity field
    divided by that of the FP64 velocity (l2_rel).  Per field, each component (and p) is
    also reported against its own maximum and 2-norm (the small components u', w carry
    only the perturbation, so their own norms are 10-20 times smaller than the speed)."""
    import numpy as np
    out = {}
    for name, x, y in zip("uvwp", a64, a32):
        den_max = max(np.abs(x).max(), 1e-300)
        den_l2 = max(np.sqrt((x * x).sum()), 1e-300)
        out[name] = {"max_rel": float(np.abs(y - x).max() / den_max),
                     "l2_rel": float(np.sqrt(((y - x) ** 2).sum()) / den_l2)}
    vmax = max(np.abs(x).max() for x in a64[:3])
    dmax = max(np.abs(y - x).max() for x, y in zip(a64[:3], a32[:3]))
    d2 = sum(((y - x) ** 2).sum() for x, y in zip(a64[:3], a32[:3]))
    v2 = sum((x * x).sum() for x in a64[:3])
    out["velocity"] = {"max_rel": float(dmax / vmax), "l2_rel": float(np.sqrt(d2 / v2))}
    return out


def measure_ensemble(n=96, steps=200, warmup=3, seed=5):
    """The ragged ensemble in FP32 storage: one HIP-graph launch per RK3 step of all
    instances (instances as parallel graph branches) vs the same kernels launched one
    instance after another on one stream, and vs a graph of batched launches (one launch
    per kernel for all instances)."""
    import torch
    import ibm_inputs as I
    from ibm_inputs import torch_gen as TG
    from paper_2506_14328_amd import IbmGrid
    cases = I.ensemble_cases(n, seed)
    dev = torch.device("cuda", 0)
    g = IbmGrid.ensemble(cases, precision="fp32")
    states = []
    for i, c in enumerate(cases):
        sdf, st = TG.make_inputs(c, dev, torch.float32)
        g.set_geometry(*sdf, inst=i)
        g.set_state(*st, inst=i)
        states.append(st)
        del sdf
    torch.cuda.synchronize()
    cells = sum(c.nx * (c.ny - 1) * c.nz for c in cases)
    res = {}
    tunings = {}
    for mode in ("sequential", "graph", "batched"):
        # the batched run takes the joint ensemble autotuner's choice (y planes per
        # momentum block and tile order, one value for all instances), the graph of
        # per-instance branches each instance's own tuning; the runs one after another
        # keep the single-grid automatic choices
        # (the batched launches also take the automatic z-FFT width and tridiagonal rows:
        # one launch runs the largest kernel variant any instance's tuning needs)
        g.tune(graph=0 if mode == "sequential" else 1, batch=1 if mode == "batched" else 0,
               momentum_planes=0, tile_order=0)
        if mode == "batched":
            g.tune(fftz_width=0, tri_rows=8)
        if mode != "sequential":
            ch = g.autotune(2)
            tunings[mode] = {"momentum_planes": ch["momentum_planes"], "tile_order": ch["tile_order"]}
        for i, st in enumerate(states):
            g.set_state(*st, inst=i)
        g.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[mode] = {"value": cells * 3 * steps / el, "ms_per_step": el / steps * 1e3}
    bad = sum(1 for i in range(n) if g.stats(inst=i)["nan_flag"])
    # whole-step fraction of the HBM peak in each mode: algorithmic bytes of one RK3 step
    # summed over the instances / measured time per step (the library's per-kernel events
    # see per-instance launches only, so the batched kernels are not timed one by one)
    n_ibm = [g.stats(inst=i)["n_ibm"] for i in range(n)]
    nb_step = 0.0
    for c, ni in zip(cases, n_ibm):
        C = c.nx * (c.ny - 1) * c.nz
        M = (c.nx // 2 + 1) * c.nz * (c.ny - 1)
        nb_step += step_bytes(C, M, 4, sum(ni), ni[0])
    step_frac = {m: round(nb_step / (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) for m, r in res.items()}
    g.close()
    return {"workload": f"ensemble_{n}_wavy_ragged", "precision": "fp32", "instances": n, "cells": cells,
            "step_algorithmic_GB": round(nb_step / 1e9, 3), "step_frac_hbm": step_frac,
            "steps": steps, "value": res["graph"]["value"], "ms_per_step": res["graph"]["ms_per_step"],
            "sequential_value": res["sequential"]["value"], "batched_graph_value": res["batched"]["value"],
            "graph_speedup": res["graph"]["value"] / res["sequential"]["value"], "instances_with_nan": bad,
            "tuning": tunings}


def measure_masked(steps=20, warmup=2, stretched=False, precision="fp64"):
    """The open channel (192 x 65 x 160, FP64) with the masked projection: continuity on
    the internal cells only, solved by conjugate gradients preconditioned with the
    full-box solve (launched eagerly, the convergence flag read every 4 iterations; then
    replayed as a graph).  stretched: on the bottom-clustered grid of spacing ratio 5.6.
    precision fp32: FP32 storage (the iteration in FP64, the FP32 full-box solve as
    preconditioner)."""
    import dataclasses
    import numpy as np
    import torch
    import ibm_inputs as I
    c, sdf, st = build_inputs("wavy_open")
    if stretched:
        c = dataclasses.replace(c, y_faces=I.bottom_tanh_faces(c.ny, c.y_lo, c.y_hi, 5.6),
                                name="wavy_open_stretched_192x65x160")
        sdf = I.make_sdf(c)
        u, v, w = I.make_initial(c, sdf)
        st = (u, v, w, np.zeros_like(u))
    c = dataclasses.replace(c, projection=1)
    g = make_grid(c, sdf, st, precision)
    tuned = g.autotune(2)
    g.set_state(*[torch.as_tensor(a).to("cuda", g.dtype) for a in st])
    g.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s = g.stats()
    g.profile(True)
    g.step(2)
    prof = g.profile_read()
    g.profile(False)
    # the same steps replayed as a HIP graph: a fixed iteration budget per solve with the
    # convergence flag tested on the device, no host synchronisation
    g.tune(graph=1)
    g.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    el_g = time.perf_counter() - t0
    sg = g.stats()
    tot = sum(v[0] for v in prof.values())
    C = c.nx * (c.ny - 1) * c.nz
    out = {"workload": c.name, "projection": "masked", "precision": precision, "value": C * 3 * steps / el,
           "ms_per_step": el / steps * 1e3, "ms_per_step_graph": el_g / steps * 1e3,
           "pcg_iterations_last_solve_graph": sg["pcg_iters"], "pcg_iterations_last_solve": s["pcg_iters"],
           "pcg_relative_residual": s["poisson_rel_residual"],
           "internal_divergence_max": s["div_max_internal_leak"],
           "kernel_time_share_pct": {k: round(100.0 * v[0] / tot, 1) for k, v in prof.items()},
           "kernel_launches_per_step": {k: v[1] // 2 for k, v in prof.items()}, "tuning": tuned}
    g.close()
    return out


def measure_moving_geometry(steps=50):
    """The 192x129x96 wavy channel whose wall translates along x (two positions half a
    cell apart, alternated): the cost of replacing the geometry before every step
    (ibm_set_geometry: tags, wall distances, lists and coefficients, S_k, all on the stream
    with no host read-back), with the library's graph replaying the steps, against the
    same steps with the geometry fixed.  FP64."""
    import numpy as np
    import torch
    import ibm_inputs as I
    c, sdf, st = build_inputs("wavy")
    g = make_grid(c, sdf, st, "fp64")
    g.autotune(2)
    g.tune(graph=1)
    # the wall moved by half a cell: sample the same wall at x - dx/2
    k = 2.0 * math.pi / c.geo_params[1]
    amp = c.geo_params[0]

    def wall(X, Y, Z):
        yw = -1.0 + amp * np.sin(k * (X - 0.5 * c.dx))
        dyw = amp * k * np.cos(k * (X - 0.5 * c.dx))
        return np.minimum((Y - yw) / np.sqrt(1.0 + dyw * dyw), 1.0 - Y)
    shifted = I._sample(c, wall)
    pos = [[torch.as_tensor(a).to("cuda") for a in sdf], [torch.as_tensor(a).to("cuda") for a in shifted]]
    g.set_geometry(*pos[1])
    g.set_geometry(*pos[0])
    g.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    t_fixed = time.perf_counter() - t0
    t0 = time.perf_counter()
    for n in range(steps):
        g.set_geometry(*pos[(n + 1) % 2])
        g.step(1)
    torch.cuda.synchronize()
    t_moving = time.perf_counter() - t0
    s = g.stats()
    g.close()
    return {"workload": "wavy_192x129x96_translating_wall", "precision": "fp64", "graph": True,
            "ms_per_step_fixed_geometry": t_fixed / steps * 1e3, "ms_per_step_moving_geometry": t_moving / steps * 1e3,
            "geometry_update_ms": (t_moving - t_fixed) / steps * 1e3, "nan_flag": s["nan_flag"]}


def measure_shard_shapes(steps=20, warmup=3):
    """One GPU's share of the 512 x 257 x 256 channel split over 8 GPUs: the 512 x 257 x 32
    z-slab that the stencil kernels would see, and a 64 x 257 x 256 grid whose 33 x-modes
    are the wave-number slab that the z-FFT and the wall-normal solve would see (one wave
    of the wall over its length, so that the geometry stays periodic).  Per-kernel averages
    from the library's HIP-event timing, FP64."""
    import math
    import numpy as np
    import torch
    import ibm_inputs as I
    out = []
    for label, over in (("z-slab of 8", dict(nz=32, lz=math.pi / 8, q_target_or_pi=2.0 * math.pi / 8,
                                            name="wavy_zslab_512x257x32")),
                        ("kx-slab of 8", dict(nx=64, lx=math.pi / 4, q_target_or_pi=2.0 * math.pi,
                                             geo_params=(0.1, math.pi / 4), name="wavy_kxslab_64x257x256"))):
        import dataclasses
        c = dataclasses.replace(I.make_case("wavy_large"), **over)
        sdf = I.make_sdf(c)
        u, v, w = I.make_initial(c, sdf)
        g = make_grid(c, sdf, (u, v, w, np.zeros_like(u)), "fp64")
        tuned = g.autotune(3)
        g.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        g.profile(True)
        g.step(5)
        prof = g.profile_read()
        g.profile(False)
        g.close()
        C = c.nx * (c.ny - 1) * c.nz
        out.append({"workload": c.name, "share": label, "precision": "fp64", "cells": C,
                    "value": C * 3 * steps / el, "ms_per_step": el / steps * 1e3,
                    "kernel_avg_us": {k: round(v[0] / v[1] * 1e3, 2) for k, v in prof.items()}, "tuning": tuned})
    return out


def cpu_baseline(name, target_s=12.0):
    """The FP64 oracle, as it stands, on the same workload: one step (untimed) when it takes
    under 2 s, then as many whole steps as fit in about target_s seconds (at least 1)."""
    import numpy as np
    from oracle.ibm_oracle import OGrid, Oracle
    c, sdf, st = build_inputs(name)
    o = Oracle(OGrid.from_case(c))
    o.set_geometry(*sdf)
    o.set_state(*st)
    t = time.perf_counter()
    o.step(1)
    first = time.perf_counter() - t
    if first > 2.0:
        # a large grid: the first step is the sample (numpy and scipy.fft need no warm-up
        # beyond their first call on small arrays, which the geometry set-up made)
        n, el = 1, first
    else:
        n = max(1, int(target_s / max(first, 1e-3)))
        t = time.perf_counter()
        o.step(n)
        el = time.perf_counter() - t
    C = c.nx * (c.ny - 1) * c.nz
    import platform
    import scipy
    model = platform.processor() or "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": C * 3 * n / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} RK3 step(s) ({3 * n} substeps) of the {c.name} workload"
                      f"{' (the first step)' if first > 2.0 else ' after 1 warm-up step'}, "
                      f"NumPy {np.__version__} / SciPy {scipy.__version__} FP64, one thread (scipy.fft "
                      f"workers=1), {model}, {os.cpu_count()} logical CPUs visible; {el:.1f} s"}


def copy_bandwidth(gib=2.0, reps=10):
    """Read + write bytes per second of the library's streaming copy kernel (16-byte vector
    loads and stores, ibm_stream_copy) over gib GiB: the practical HBM ceiling of a kernel
    that moves every byte once.  Timed with HIP events on torch's current stream, which is
    the stream the copy is enqueued on."""
    import torch
    from paper_2506_14328_amd import stream_copy
    n = int(gib * (1 << 30) // 8)
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    stream_copy(y, x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        stream_copy(y, x)
    e1.record()
    e1.synchronize()
    gbs = 2.0 * n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    assert bool((y == 1.0).all())
    del x, y
    torch.cuda.empty_cache()
    return gbs


def stream_mix_bandwidth(cells, elem_bytes, reps=5):
    """Bytes per second of the library's stream-mix kernel (ibm_stream_mix) with the
    momentum kernel's stream counts over the three RK3 stages, arrays of one field each:
    stage 1 reads 5 fields and writes 7, stage 2 reads 8 and writes 7, stage 3 reads 8 and
    writes 4 (the tag byte left out).  Total bytes / total time of the three: the practical
    HBM ceiling of a kernel with that mix of read and write streams."""
    import torch
    from paper_2506_14328_amd import stream_mix
    n = cells * elem_bytes // 8
    arrs = [torch.full((n,), 1.0, dtype=torch.float64, device="cuda") for _ in range(15)]
    mixes = ((5, 7), (8, 7), (8, 4))
    for ns, nd in mixes:
        stream_mix(arrs[8:8 + nd], arrs[:ns])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        for ns, nd in mixes:
            stream_mix(arrs[8:8 + nd], arrs[:ns])
    e1.record()
    e1.synchronize()
    nbytes = reps * sum(ns + nd for ns, nd in mixes) * n * 8
    gbs = nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9
    assert bool((arrs[8] == 8.0).all())
    del arrs
    torch.cuda.empty_cache()
    return gbs


def stream_table(cells=512 * 256 * 256, reps=10):
    """Read + write bytes per second of ibm_stream_copy and of ibm_stream_mix for several
    (reads, writes) stream counts, FP64 arrays of `cells` values (and FP32-sized arrays for
    the momentum kernel's mix), HIP events on torch's current stream."""
    import torch
    from paper_2506_14328_amd import stream_copy, stream_mix
    rows = []

    def timed(fn, nbytes):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    arrs = [torch.full((cells,), 1.0, dtype=torch.float64, device="cuda") for _ in range(16)]
    gbs = timed(lambda: stream_copy(arrs[8], arrs[0]), 2 * cells * 8)
    rows.append({"kernel": "stream_copy", "reads": 1, "writes": 1, "GBs": round(gbs, 1)})
    for ns, nd in ((1, 1), (2, 2), (4, 4), (8, 1), (1, 7), (5, 7), (8, 7), (8, 4)):
        gbs = timed(lambda: stream_mix(arrs[8:8 + nd], arrs[:ns]), (ns + nd) * cells * 8)
        rows.append({"kernel": "stream_mix", "reads": ns, "writes": nd, "GBs": round(gbs, 1)})
    del arrs
    torch.cuda.empty_cache()
    for eb in (8, 4):
        rows.append({"kernel": "stream_mix", "mix": "momentum stages (5+7, 8+7, 8+4)",
                     "array_bytes": cells * eb, "GBs": round(stream_mix_bandwidth(cells, eb), 1)})
    for r in rows:
        r["frac_of_peak"] = round(r["GBs"] / HBM_PEAK_GBS, 4)
        print(json.dumps(r), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    torch.cuda.set_device(0)
    if a.stream_table:
        stream_table()
        return
    if a.only_form:
        if a.only_form == "ensemble":
            res = measure_ensemble(steps=a.steps)
        elif a.only_form == "masked":
            res = measure_masked()
        elif a.only_form == "moving":
            res = measure_moving_geometry()
        else:
            res = measure_shard_shapes()
        print(json.dumps(res), flush=True)
        return

    if a.copy_calibration_mb > 0:
        from paper_2506_14328_amd import stream_copy
        n = int(a.copy_calibration_mb * (1 << 20) // 8)
        # the library's streaming copy (kernel k_stream_copy), whose bytes are known exactly
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            stream_copy(y, x)
        torch.cuda.synchronize()
        print(f"copy calibration (k_stream_copy): {n * 8} bytes read, {n * 8} bytes written per launch",
              flush=True)

    inputs = build_inputs(a.workload)
    if a.projection == "masked":
        import dataclasses
        inputs = (dataclasses.replace(inputs[0], projection=1),) + tuple(inputs[1:])
    fixed = {k: int(v) for k, v in (kv.split("=") for kv in a.tuning.split(",") if kv)} if a.tuning else None
    r = measure(a.workload, a.precision, a.steps, a.warmup, inputs=inputs, tuning=fixed)
    if a.profile_only:
        print(json.dumps({"workload": r["case"].name, "ms_per_step": r["ms_per_step"], "kernel": r["kernel"],
                          "kernel_avg_us": r["kernel_avg_us"]}), flush=True)
        return
    c = r["case"]
    traffic = load_traffic(r["kernel"], c.name, a.precision)
    roof = {"bound": "hbm", "achieved": round(r["achieved_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": r["kernel"], "kernel_avg_us": round(r["kernel_avg_us"], 2),
            "algorithmic_bytes_per_launch": int(r["kernel_bytes"]),
            "step_algorithmic_GBs": round(r["step_gbs"], 1)}
    roof["measured_copy_GBs"] = round(copy_bandwidth(), 1)   # practical ceiling on this device
    if r["kernel"] == "momentum":
        # the ceiling of a kernel with the momentum kernel's read and write streams
        mix = stream_mix_bandwidth(r["cells"], 8 if a.precision == "fp64" else 4)
        roof["measured_stream_mix_GBs"] = round(mix, 1)
        roof["frac_of_stream_mix"] = round(r["achieved_gbs"] / mix, 4)
    out = {"metric": METRIC, "value": r["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if a.precision == "fp64" else "f32",
           "data": "synthetic (seeded sinusoidal-wall channel, laminar + solenoidal perturbation)",
           "config": {"workload": c.name, "grid_faces": [c.nx, c.ny, c.nz], "cells": r["cells"],
                      "projection": "masked" if c.projection == 1 else "full box",
                      "precision": a.precision, "Re_bulk": round(1.0 / c.nu), "dt": c.dt,
                      "forcing": "constant flow rate", "ibm_point_fraction": round(r["ibm_fraction"], 4)},
           "roofline": roof, "kernel_time_share_pct": r["shares"], "tuning": r["tuning"]}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.workload)
    if not a.no_forms:
        import torch
        forms = []
        off = measure(a.workload, a.precision, a.steps, a.warmup, ibm=False, inputs=inputs)
        forms.append(dict(_form(off, a.precision), ibm="off (staircase)",
                          ibm_cost_pct=round(100.0 * (r["ms_per_step"] / off["ms_per_step"] - 1.0), 1)))
        # large sinusoidal channel in FP32 storage: 200 steps from the same start as a
        # 200-step FP64 run, error of the FP32 state against the FP64 one
        big = inputs if a.workload == "wavy_large" and a.projection == "full" else build_inputs("wavy_large")
        r64 = measure("wavy_large", "fp64", 200, 0, inputs=big, keep_state=True)
        st64 = r64["state"]
        del r64
        r32 = measure("wavy_large", "fp32", 200, 0, inputs=big, keep_state=True)
        err = precision_errors(st64, r32["state"])
        forms.append(dict(_form(r32, "fp32"), error_vs_fp64_after_200_steps=err))
        del big, r32, st64
        # the 192x129x96 channel (its working set fits the 256 MB Infinity Cache)
        small = build_inputs("wavy")
        for prec in ("fp64", "fp32"):
            forms.append(_form(measure("wavy", prec, 300, 3, inputs=small), prec))
        del small
        # complex geometry: union of 64 ellipsoids, 300 steps
        from ibm_inputs import torch_gen as TG
        import ibm_inputs as I
        ce = I.make_case("ellipsoids")
        sdf_e, st_e = TG.make_inputs(ce, torch.device("cuda", 0), torch.float64)
        inp_e = (ce, sdf_e, st_e)
        for prec in ("fp64", "fp32"):
            re_ = measure("ellipsoids", prec, 300, 3, inputs=inp_e)
            forms.append(dict(_form(re_, prec), ibm_point_fraction=round(re_["ibm_fraction"], 4)))
        del sdf_e, st_e, inp_e
        torch.cuda.empty_cache()
        # open channel over an undulated bottom, free-slip top (192 x 65 x 160), 300 steps
        inp_o = build_inputs("wavy_open")
        ro = measure("wavy_open", "fp64", 300, 3, inputs=inp_o)
        forms.append(dict(_form(ro, "fp64"), top="free-slip", ibm_point_fraction=round(ro["ibm_fraction"], 4)))
        del inp_o
        # the same open channel on a wall-normal grid clustered towards the bottom with the
        # largest/smallest spacing ratio of the paper's 64-point grid (5.6), FP64, 300 steps
        import dataclasses
        import numpy as np
        import ibm_inputs as I
        c0 = I.make_case("wavy_open")
        cso = dataclasses.replace(c0, y_faces=I.bottom_tanh_faces(c0.ny, c0.y_lo, c0.y_hi, 5.6),
                                  name="wavy_open_stretched_192x65x160")
        sdf_so = I.make_sdf(cso)
        uo, vo, wo = I.make_initial(cso, sdf_so)
        rso = measure("wavy_open", "fp64", 300, 3, inputs=(cso, sdf_so, (uo, vo, wo, np.zeros_like(uo))))
        forms.append(dict(_form(rso, "fp64"), top="free-slip", y_faces="bottom-clustered tanh, spacing ratio 5.6",
                          ibm_point_fraction=round(rso["ibm_fraction"], 4)))
        del sdf_so, uo, vo, wo
        # the wavy channel on a stretched wall-normal grid (faces clustered towards both box
        # walls, tanh with gamma 1.2: spacing ratio 3.3), FP64, 300 steps
        import dataclasses
        import numpy as np
        import ibm_inputs as I
        cw = I.make_case("wavy")
        cs = dataclasses.replace(cw, y_faces=I.tanh_faces(cw.ny, cw.y_lo, cw.y_hi, 1.2),
                                 name="wavy_stretched_192x129x96")
        sdf_s = I.make_sdf(cs)
        us_, vs_, ws_ = I.make_initial(cs, sdf_s)
        rs = measure("wavy", "fp64", 300, 3, inputs=(cs, sdf_s, (us_, vs_, ws_, np.zeros_like(us_))))
        dyc = np.diff(np.asarray(cs.y_faces))
        forms.append(dict(_form(rs, "fp64"), y_faces="tanh, gamma 1.2",
                          spacing_ratio=round(float(dyc.max() / dyc.min()), 2),
                          ibm_point_fraction=round(rs["ibm_fraction"], 4)))
        del sdf_s, us_, vs_, ws_
        forms.append(measure_masked())
        forms.append(measure_masked(stretched=True))
        forms.append(measure_masked(precision="fp32"))
        forms.append(measure_moving_geometry())
        forms.extend(measure_shard_shapes())
        forms.append(measure_ensemble())
        out["forms"] = forms
    print(json.dumps(out), flush=True)


def _form(r, prec):
    return {"workload": r["case"].name, "precision": prec, "value": r["value"], "ms_per_step": r["ms_per_step"],
            "dominant_kernel": r["kernel"], "kernel_frac_hbm": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
            "step_algorithmic_GBs": round(r["step_gbs"], 1),
            "step_frac_hbm": round(r["step_gbs"] / HBM_PEAK_GBS, 4), "tuning": r["tuning"]}


if __name__ == "__main__":
    main()
