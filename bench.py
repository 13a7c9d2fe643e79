"""Benchmark: cell-updates/s of the full RANS step (incl. the pressure solve).

Workload (default): the 512x512x128 city (1 m cells, 200 buildings and 400
porous trees drawn from the seeded generator, log-law inflow of 6 m/s at
10 m from a seeded random direction), FP32 with FP64 reductions,
multigrid-preconditioned CG to a relative residual of 1e-6.  Inputs are
resident on the GPU before the timed region.  --workload C1 selects the
256x256x64 city.

Prints one JSON line:  value = cells x steps / seconds over K timed steps
(bracketed by device synchronisation), the roofline figure of the kernel
with the largest share of the step time, measured live with HIP events
around each of its launches, the whole step's HBM traffic from the
committed counter summary, and the FP64 oracle timed on this host on a
bounded sample of the same workload (before the GPU is touched).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Profiling helpers (the commands are recorded in the files they write):
    python bench.py --traffic-probe [--workload W]
        a few steps of the workload, then a plain copy of COPY_BYTES: the
        program run under rocprofv3 --pmc FETCH_SIZE and, separately,
        --pmc WRITE_SIZE (csv output under <dir>/fetch and <dir>/write)
    python bench.py --traffic-summary <dir> [--workload W]
        HBM bytes per launch of each kernel from those two runs, scaled by
        what the counters read for the copy, into
        profiles/traffic_<kernel>_<grid>.json
    python bench.py --precond-study
        the pressure system of the workload solved with each preconditioner
        (iterations and solve time per case, one JSON line each)
    python bench.py --stats-summary <dir> --command "<rocprofv3 command>" --stats-out <name>
        profiles/<name> from a rocprofv3 --kernel-trace --stats csv run
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per cell of one launch (FP32; compulsory reads and
# writes of the arrays each kernel streams).  Cells = nx * ny * nz.
ALG_BYTES_PER_CELL = {
    "cg_Ad": 16.0,        # read z, d_old; write d, q
    "cg_axpy": 24.0,      # read x, r, d, q; write x, r
    "mg_up0": 8.5,        # read r, the level-1 correction (1/8); write z
    "mg_down0": 4.5,      # read r; write the level-1 residual (1/8)
    "mg_update0": 24.5,   # read x, r, d, q; write x, r and the level-1 residual (1/8)
    "mg_rupd0": 12.5,     # marching form: read r, q; write r and the level-1 residual (1/8)
    "cg_xupd": 12.0,      # read x, d; write x (beside the coarse levels, with the marching form)
    "cg_init": 20.0,      # read u*, v*, w*, p; write r
    "advect_fwd": 24.0,   # read u, v, w; write the forward-traced u, v, w
    "advect_corr": 36.0,  # read u, v, w and the traced fields; write u, v, w
    "diffuse": 28.0,      # read u, v, w, nu_t; write u, v, w
    "drag": 28.0,         # read u, v, w, drag coefficient; write u, v, w
    "project": 28.0,      # read u*, v*, w*, p; write u, v, w
    "turbulence": 32.0,   # read u, v, w, k, omega; write k, omega, nu_t
}

# Per step outside the pressure iterations: the face and cell kernels and
# the right-hand side; per CG iteration: A d, the update and one multigrid
# application (its coarse levels add about 1/7 of the level-0 kernels).
STEP_FIXED_KERNELS = ("advect_fwd", "advect_corr", "diffuse", "drag", "project", "turbulence", "cg_init")
ALG_FIXED_PER_CELL = sum(ALG_BYTES_PER_CELL[k] for k in STEP_FIXED_KERNELS)
# (the marching form's split into mg_rupd0 + cg_xupd moves the same bytes as mg_update0)
ALG_ITER_PER_CELL = (ALG_BYTES_PER_CELL["cg_Ad"] + ALG_BYTES_PER_CELL["mg_update0"] - ALG_BYTES_PER_CELL["mg_down0"] +
                     (ALG_BYTES_PER_CELL["mg_up0"] + ALG_BYTES_PER_CELL["mg_down0"]) * 8.0 / 7.0)
STEP_PREFIXES = ("k_advect_", "k_diffuse", "k_drag", "k_project", "k_turbulence", "k_cg_init", "k_cg_start")
ITER_PREFIXES = ("k_cg_Ad", "k_cg_axpy", "k_cg_xupd", "k_mg_", "k_cg_precond", "k_ai2_", "k_cg_status")

# Kernels of the library by their profiler names (first match wins) and
# the names the kernel timer and ALG_BYTES_PER_CELL use.
PROFILE_NAMES = [
    ("k_cg_Ad<", "cg_Ad"),
    ("k_mg_axpy<", "cg_axpy"),
    ("k_cg_axpy<", "cg_axpy"),
    ("k_mg_upsmooth<true", "mg_up0"),
    ("k_mg_upsmooth_march<", "mg_up0"),
    ("k_mg_restrict<true", "mg_update0"),
    ("k_mg_update_march<true", "mg_rupd0"),
    ("k_cg_xupd<", "cg_xupd"),
    ("k_mg_update_march<false", "mg_down0"),
    ("k_cg_init<", "cg_init"),
    ("k_advect_fwd<", "advect_fwd"),
    ("k_advect_fwd32<", "advect_fwd"),
    ("k_advect_corr<", "advect_corr"),
    ("k_advect_corr32<", "advect_corr"),
    ("k_diffuse<", "diffuse"),
    ("k_drag<", "drag"),
    ("k_project<", "project"),
    ("k_turbulence<", "turbulence"),
]

# Calibration copy of the counter runs: bytes read (and written) once.
COPY_BYTES = 1 << 30

# Grid tag of each step workload (names of the counter and kernel summaries).
GRID_TAG = {"C1": "256x256x64", "C2": "512x512x128", "slab": "64x512x128", "CP": "450x300x40"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name="C2"):
    """C2: the 512x512x128 city (the default).  C1: the 256x256x64 city.
    slab: one GPU's share of C2 split eight ways along x (64x512x128, the
    first slab of C2's layout, with the domain's own side conditions where
    a split run would exchange halos)."""
    from uf_layouts import preset, preset_porosity
    if name == "slab":
        p = preset("C2")
        phi, cfg = preset_porosity(p)
        nx = cfg["nx"] // 8
        phi = phi[:nx].copy()
        cfg = dict(cfg, nx=nx)
        p = dict(p, workload="64x512x128 x-slab (1/8) of " + p["workload"])
        return p, phi, cfg
    p = preset(name)
    phi, cfg = preset_porosity(p)
    return p, phi, cfg


def copy_ceiling_gbs(torch, nbytes=1 << 30, reps=5):
    """Read + write bandwidth of a plain device copy (the practical ceiling
    of the streaming kernels)."""
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del x, y
    return gbs


def traffic_for(kernel, tag):
    """HBM bytes per launch from the committed counter summary of this kernel
    (profiles/traffic_<kernel>_<tag>.json), or None when there is none or
    the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, tag))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != sources_hash(kernel):
        return None
    return rec.get("bytes_per_launch")


def step_traffic(iters_per_step, ms_per_step, ncells, tag):
    """HBM bytes of a whole step from the committed counter summary
    (profiles/traffic_step_<tag>.json) at this iteration count, with the
    bandwidth they imply over the step's wall time; None when absent or
    stale."""
    path = os.path.join(ROOT, "profiles", "traffic_step_%s.json" % tag)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != sources_hash():
        return None
    meas = rec["bytes_fixed_per_step"] + iters_per_step * rec["bytes_per_cg_iteration"]
    alg = (ALG_FIXED_PER_CELL + iters_per_step * ALG_ITER_PER_CELL) * ncells
    gbs = meas / (ms_per_step / 1e3) / 1e9
    return {"bytes_per_step": meas, "alg_bytes_per_step": alg, "achieved_GBs": gbs,
            "alg_GBs": alg / (ms_per_step / 1e3) / 1e9, "frac": gbs / HBM_PEAK_GBS,
            "source": "profiles/traffic_step_%s.json" % tag}


# Source files that hold each measured kernel's device code (with the
# device headers every kernel includes): a counter record is stale when
# these change, and only then.
KERNEL_FILES = {
    "advect_fwd": ["k_momentum.hip", "face_ops.h"], "advect_corr": ["k_momentum.hip", "face_ops.h"],
    "diffuse": ["k_momentum.hip", "face_ops.h"], "drag": ["k_momentum.hip", "face_ops.h"],
    "project": ["k_momentum.hip", "face_ops.h"], "turbulence": ["k_cells.hip", "turb_model.h"],
    "cg_Ad": ["k_pressure.hip"], "cg_axpy": ["k_pressure.hip"], "cg_init": ["k_pressure.hip"],
    "mg_up0": ["k_mg.hip"], "mg_down0": ["k_mg.hip"], "mg_update0": ["k_mg.hip"], "mg_rupd0": ["k_mg.hip"],
    "cg_xupd": ["k_mg.hip"],
}
DEVICE_HEADERS = ["uf_device.h", "pressure_common.h"]


def sources_hash(kernel=None):
    """sha256 of the sources of one kernel (None: of every step kernel)."""
    files = KERNEL_FILES.get(kernel) or sorted({f for v in KERNEL_FILES.values() for f in v})
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2204_01117_amd", "csrc")
    for name in sorted(set(files) | set(DEVICE_HEADERS)):
        h.update(name.encode())
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()


def profile_name(kernel_name):
    for pat, name in PROFILE_NAMES:
        if pat in kernel_name:
            return name
    return None


def _counter_rows(run_dir):
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no *counter_collection.csv under %s" % run_dir)
    for f in files:
        for row in csv.DictReader(open(f)):
            yield row


def _dispatches(run_dir, counter):
    """(kernel name, grid size, value) of every dispatch for one counter."""
    acc = {}
    for row in _counter_rows(run_dir):
        if row.get("Counter_Name") != counter:
            continue
        key = (row["Kernel_Name"], int(row.get("Grid_Size") or 0), row.get("Dispatch_Id"))
        acc[key] = acc.get(key, 0.0) + float(row["Counter_Value"])
    return [(k[0], k[1], v) for k, v in acc.items()]


def _per_kernel(disp):
    """Average per dispatch by (kernel name, grid size).  Dispatches below 5%
    of the largest of their group are left out: launches that returned at
    once (a step's projection and k-omega update enqueued before the solve's
    end was known skip when the solve went on, and run again after it)."""
    per = {}
    for name, grid, v in disp:
        per.setdefault((name, grid), []).append(v)
    out = {}
    for k, v in per.items():
        top = max(v)
        kept = [x for x in v if x >= 0.05 * top] if top > 0 else v
        out[k] = sum(kept) / len(kept)
    return out


def _copy_calibration(disp):
    """Average counter value of the calibration copies: the copy-kernel
    dispatches within 10% of the largest one (smaller runtime copies of the
    set-up are left out)."""
    vals = [v for name, _, v in disp if "copy" in name.lower()]
    if not vals:
        raise SystemExit("no copy kernel in the counter runs")
    top = max(vals)
    big = [v for v in vals if v >= 0.9 * top]
    return sum(big) / len(big), len(big)


def traffic_probe(name):
    """The program profiled for the traffic counters: the workload for a
    few steps, then a plain device copy of COPY_BYTES (the calibration)."""
    import torch
    import paper_2204_01117_amd as U
    _, phi, cfg = workload(name)
    g = U.Grid(cfg, device="cuda:0")
    g.set_porosity(torch.as_tensor(phi))
    g.step(3)
    g.step(3)
    torch.cuda.synchronize()
    # two streaming kernels of known footprint besides the copy: the layout
    # conversion (compact <-> padded, 8 B per cell each way) and the 7-point
    # operator (read x, write A x: 8 B per cell)
    n = (cfg["nx"], cfg["ny"], cfg["nz"])
    xin = torch.rand(n, dtype=torch.float32, device="cuda:0")
    g.apply_operator(0, xin)
    torch.cuda.synchronize()
    g.close()
    del xin
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    log("traffic probe done: 6 steps, one operator application, 3 copies of %d bytes" % COPY_BYTES)


def traffic_summary(run_dir, command, out_dir=None, name="C2"):
    """Counter records of every measured kernel and of the whole step of
    workload ``name`` from the FETCH_SIZE and WRITE_SIZE runs under run_dir,
    written to out_dir (default profiles/)."""
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    tag = GRID_TAG[name]
    _, _, wcfg = workload(name)
    ncell = wcfg["nx"] * wcfg["ny"] * wcfg["nz"]
    fd = _dispatches(os.path.join(run_dir, "fetch"), "FETCH_SIZE")
    wd = _dispatches(os.path.join(run_dir, "write"), "WRITE_SIZE")
    c_fetch, n_fetch = _copy_calibration(fd)
    c_write, n_write = _copy_calibration(wd)
    f_fetch = c_fetch * 1024.0 / COPY_BYTES
    f_write = c_write * 1024.0 / COPY_BYTES
    fetch, write = _per_kernel(fd), _per_kernel(wd)
    # one entry per timer name: the group with the largest grid (the finest
    # level for the multigrid kernels)
    best = {}
    for (name, grid) in fetch:
        bn = profile_name(name)
        if bn is None or (name, grid) not in write:
            continue
        if bn not in best or grid > best[bn][1]:
            best[bn] = (name, grid)
    # the first restriction of a solve, when tiled: the largest tiled restriction
    if "mg_down0" not in best:
        cands = [(n, gr) for (n, gr) in fetch if "k_mg_restrict<false" in n and (n, gr) in write]
        if cands:
            best["mg_down0"] = max(cands, key=lambda k: k[1])
    out = {}
    for bn, key in best.items():
        fb = fetch[key] * 1024.0 / f_fetch
        wb = write[key] * 1024.0 / f_write
        out[bn] = {
            "kernel": bn, "profiler_name": key[0].split("(")[0], "grid_size": key[1], "workload": tag,
            "bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
            "fetch_kib_raw": fetch[key], "write_kib_raw": write[key],
            "calibration": {"copy_bytes": COPY_BYTES, "copies": [n_fetch, n_write],
                            "fetch_kib_raw": c_fetch, "write_kib_raw": c_write,
                            "fetch_factor": f_fetch, "write_factor": f_write},
            "alg_bytes_per_launch": ALG_BYTES_PER_CELL[bn] * ncell,
            "source_sha256": sources_hash(bn),
            "command": command,
        }
    # the whole step: every dispatch of the step's kernels, split into the
    # part per step and the part per CG iteration
    def short(n):
        return n.split("(")[0].replace("void ", "").replace("uf::", "")
    tot = {"step": 0.0, "iter": 0.0}
    steps = iters = 0
    for disp, factor in ((fd, f_fetch), (wd, f_write)):
        for name, _, v in disp:
            n = short(name)
            if n.startswith(STEP_PREFIXES):
                tot["step"] += v * 1024.0 / factor
            elif n.startswith(ITER_PREFIXES):
                tot["iter"] += v * 1024.0 / factor
    for name, _, _ in fd:
        n = short(name)
        steps += n.startswith("k_advect_fwd")
        iters += n.startswith("k_cg_Ad")
    step_rec = {
        "workload": tag, "steps": steps, "cg_iterations": iters,
        "bytes_fixed_per_step": tot["step"] / max(steps, 1),
        "bytes_per_cg_iteration": tot["iter"] / max(iters, 1),
        "alg_bytes_fixed_per_step": ALG_FIXED_PER_CELL * ncell,
        "alg_bytes_per_cg_iteration": ALG_ITER_PER_CELL * ncell,
        "calibration": {"fetch_factor": f_fetch, "write_factor": f_write},
        "source_sha256": sources_hash(), "command": command,
    }
    # the copy calibration applied to the known-footprint kernels of the
    # probe (8 B per cell each): how far it transfers to other patterns
    # (per kernel, the launch that moved the most: the probe's full-grid one)
    checks = {}
    for (kname, grid), fv in fetch.items():
        short_name = kname.split("(")[0].replace("void ", "").replace("uf::", "")
        if not short_name.startswith(("k_pack<", "k_apply<")) or (kname, grid) not in write:
            continue
        meas = fv * 1024.0 / f_fetch + write[(kname, grid)] * 1024.0 / f_write
        foot = 8.0 * ncell
        if short_name not in checks or meas > checks[short_name]["bytes_per_launch"]:
            checks[short_name] = {"bytes_per_launch": meas, "footprint_bytes": foot, "ratio": meas / foot,
                                  "grid_size": grid}
    step_rec["calibration_checks"] = checks
    for k, v in checks.items():
        log("calibration check %-36s counters/footprint %.3f" % (k, v["ratio"]))
    with open(os.path.join(out_dir, "traffic_step_%s.json" % tag), "w") as f:
        json.dump(step_rec, f, indent=1)
        f.write("\n")
    log("step traffic: %.3e B fixed per step (alg %.3e), %.3e B per CG iteration (alg %.3e)"
        % (step_rec["bytes_fixed_per_step"], step_rec["alg_bytes_fixed_per_step"],
           step_rec["bytes_per_cg_iteration"], step_rec["alg_bytes_per_cg_iteration"]))
    for bn, rec in out.items():
        path = os.path.join(out_dir, "traffic_%s_%s.json" % (bn, tag))
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
        log("%-12s traffic %.3e B/launch (alg %.3e, ratio %.2f), fetch factor %.3f write factor %.3f"
            % (bn, rec["bytes_per_launch"], rec["alg_bytes_per_launch"],
               rec["bytes_per_launch"] / rec["alg_bytes_per_launch"], f_fetch, f_write))
    return out, step_rec


def stats_summary(run_dir, command, out_name="kernels_256x256x64.md",
                  title="Kernel time, 256x256x64 city workload (FP32, multigrid-preconditioned CG)"):
    files = glob.glob(os.path.join(run_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit("no *kernel_stats.csv under %s" % run_dir)
    rows = list(csv.DictReader(open(files[0])))
    traces = glob.glob(os.path.join(run_dir, "**", "*kernel_trace.csv"), recursive=True)
    lines = ["# " + title, "",
             "Command (from the repository root):", "", "    " + command, ""]
    if traces:
        # from the trace, without the launches that returned at once (under 15%
        # of their kernel's median: CG iterations enqueued past convergence,
        # and a step's projection and k-omega update enqueued before the
        # solve's end was known, which skip when it went on)
        per = {}
        for r in csv.DictReader(open(traces[0])):
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("uf::", "")
            per.setdefault(name, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        kept, skipped = {}, 0
        for name, d in per.items():
            med = sorted(d)[len(d) // 2]
            k = [x for x in d if x >= 0.15 * med]
            skipped += len(d) - len(k)
            kept[name] = k
        total = sum(sum(k) for k in kept.values())
        lines += ["Launches that returned at once (left out): %d." % skipped, "",
                  "| kernel | calls | avg us | total ms | % |", "|---|---:|---:|---:|---:|"]
        for name, d in sorted(kept.items(), key=lambda kv: -sum(kv[1])):
            lines.append("| `%s` | %d | %.2f | %.3f | %.1f |" % (name, len(d), sum(d) / len(d) / 1e3, sum(d) / 1e6,
                                                                100.0 * sum(d) / total))
    else:
        lines += ["| kernel | calls | avg us | total ms | % |", "|---|---:|---:|---:|---:|"]
        for r in rows:
            name = r["Name"].split("(")[0].replace("void ", "").replace("uf::", "")
            lines.append("| `%s` | %s | %.2f | %.3f | %.1f |" % (
                name, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6,
                float(r["Percentage"])))
    if traces:
        groups = {}
        for r in csv.DictReader(open(traces[0])):
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("uf::", "")
            threads = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            wg = int(r["Workgroup_Size_X"]) * int(r["Workgroup_Size_Y"]) * int(r["Workgroup_Size_Z"])
            key = (name, threads // max(1, wg))
            groups.setdefault(key, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        lines += ["", "By launch shape (the multigrid kernels run once per level):", "",
                  "| kernel | blocks | calls | avg us | total ms |", "|---|---:|---:|---:|---:|"]
        for (name, blocks), d in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:24]:
            lines.append("| `%s` | %d | %d | %.2f | %.3f |" % (name, blocks, len(d), sum(d) / len(d) / 1e3,
                                                               sum(d) / 1e6))
    path = os.path.join(ROOT, "profiles", out_name)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    log("wrote", path)


def precond_study():
    """Pressure solves for each preconditioner (the paper's comparison, Sec. 3
    and its Tables 2-3) on the 256x256x64 system and on the 2-D 128x192
    system of Table 3 (inlet and outlet across x, walls and slip sides
    elsewhere): seeded normal right-hand side, zero initial guess, the
    paper's stopping rule (M^-1 r . r / ||b||^2 < 1e-5) and the default one
    (||r|| <= 1e-6 ||b||).  One JSON line per case: iterations and GPU time
    of the solve."""
    import numpy as np
    import torch
    import paper_2204_01117_amd as U
    from uf_layouts import default_config
    from uf_layouts.configs import PC_NONE, PC_JACOBI, PC_AI1, PC_AI2, PC_MG, BC_INLET, BC_OUTLET, BC_WALL, BC_SLIP
    _, _, cfg3 = workload("C1")
    cfg2 = default_config(128, 192, 1, 1.0, dtype="f32",
                          bc=[BC_INLET, BC_OUTLET, BC_WALL, BC_WALL, BC_SLIP, BC_SLIP])
    cases = [("CG", PC_NONE, 1.6), ("Jacobi", PC_JACOBI, 1.6), ("AI1", PC_AI1, 1.0), ("AI1", PC_AI1, 1.6),
             ("AI1", PC_AI1, 1.8), ("AI2", PC_AI2, 1.0), ("AI2", PC_AI2, 1.6), ("AI2", PC_AI2, 1.8),
             ("MG", PC_MG, 1.6)]
    for cfg, crit, tol in ((cfg2, 1, 1e-5), (cfg3, 1, 1e-5), (cfg3, 0, 1e-6)):
        shape = (cfg["nx"], cfg["ny"], cfg["nz"])
        b = torch.tensor(np.random.default_rng(7).normal(size=shape), dtype=torch.float32, device="cuda:0")
        for name, pc, om in cases:
            g = U.Grid(dict(cfg, precond=pc, ai_omega=om, cg_criterion=crit, cg_tol=tol, cg_maxit=20000),
                       device="cuda:0")
            g.pressure_solve(b)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            _, st = g.pressure_solve(b)
            e1.record()
            torch.cuda.synchronize()
            g.close()
            print(json.dumps({"precond": name, "omega": om if pc in (PC_AI1, PC_AI2) else None,
                              "criterion": "paper (Mr.r/|b|^2 < 1e-5)" if crit else "|r| <= 1e-6 |b|",
                              "iterations": st["cg_iters"], "ms": e0.elapsed_time(e1),
                              "converged": st["converged"], "grid": list(shape)}), flush=True)


# The oracle's sample for the CPU baseline: one complete oracle step on x-slab
# s (of 8) of the workload, a 1/8 share of its cells with the domain's own
# side conditions (as the slab workload).  Set in the parent before the
# worker processes are forked, so that they share it.
_SAMPLE = {}


def _slab(phi, cfg, s):
    nx = cfg["nx"] // 8
    return phi[s * nx:(s + 1) * nx].copy(), dict(cfg, nx=nx, dtype="f64")


def _oracle_slab_step(s, barrier=None):
    """Set up the oracle on slab s, wait at the barrier (so that concurrent
    workers time the same interval), time one step; returns seconds."""
    from threadpoolctl import threadpool_limits
    from oracle import OracleGrid
    with threadpool_limits(1):
        phi, cfg = _slab(_SAMPLE["phi"], _SAMPLE["cfg"], s % 8)
        og = OracleGrid(cfg)
        og.set_porosity(phi)
        if barrier is not None:
            barrier.wait()
        t0 = time.perf_counter()
        og.step(1)
        return time.perf_counter() - t0


def _slab_worker(s, q):
    try:
        q.put(_oracle_slab_step(s, _SAMPLE["barrier"]))
    except Exception:
        q.put(None)
        raise


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, phi, cfg):
    """The FP64 oracle, as it is, on a bounded sample of the workload: one
    complete step (advection, diffusion, drag, the exact pressure solve and
    projection, k-omega) on a 1/8 x-slab of the grid, timed on one core, then
    on every core of this host's share at once (one process per core, each
    stepping a slab; the oracle's NumPy/SciPy work is single-threaded, so
    processes are how it uses several cores).  Runs before the GPU is
    touched (the workers are forked)."""
    import multiprocessing as mp
    _SAMPLE.update(phi=phi, cfg=cfg)
    ncell = (cfg["nx"] // 8) * cfg["ny"] * cfg["nz"]
    t1 = _oracle_slab_step(0)
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    # at most 16 workers (one GPU's share of a host), each holding about
    # 3 GB for a 64x512x128 slab
    nproc = max(1, min(ncpu, 16))
    ctx = mp.get_context("fork")
    _SAMPLE["barrier"] = ctx.Barrier(nproc)      # inherited by the forked workers
    q = ctx.Queue()
    procs = [ctx.Process(target=_slab_worker, args=(s, q)) for s in range(nproc)]
    for pr in procs:
        pr.start()
    times = [q.get() for _ in procs]
    for pr in procs:
        pr.join()
    if any(t is None for t in times):
        raise RuntimeError("an oracle worker of the CPU baseline failed")
    t_all = max(times)
    return {
        "value": nproc * ncell / t_all, "unit": "cell-updates/s", "cores": nproc, "kind": "oracle",
        "sample": ("one complete oracle step (FP64 NumPy/SciPy; exact fast-diagonalisation pressure solve) on a "
                   "%dx%dx%d x-slab (1/8) of the %s workload per process, %d processes at once (one per core); "
                   "%.1f s per slab step on all cores, %.1f s on one core alone"
                   % (cfg["nx"] // 8, cfg["ny"], cfg["nz"], GRID_TAG.get(name, name), nproc, t_all, t1)),
        "seconds_per_step": t_all * 8.0 / nproc,
        "one_core": {"value": ncell / t1, "seconds_per_slab_step": t1, "seconds_per_step": t1 * 8.0},
        "host": {"nproc": ncpu, "cpu_model": _cpu_model()},
    }


FP64_PEAK_TFLOPS = 78.6
VOX_FLOPS_PER_TEST = 11   # FP64 operations of one line/triangle test (two
                          # differences, the scaled u and v numerators, u + v)


def voxelize_bench(steps, warmup, with_cpu):
    """The mesh voxelizer on the 256x256x64 city (40 box buildings, 60 trees
    as 16-sided prisms, 4x4x4 sub-samples per cell): wall time per call and
    the ray-casting kernel against the FP64 ALU roof."""
    import numpy as np
    import torch
    import paper_2204_01117_amd as U
    from uf_layouts import preset, random_city
    from uf_layouts.meshes import city_meshes
    p = preset("C1")
    cfg, lay = p["config"], p["layout"]
    n, h, sub = (cfg["nx"], cfg["ny"], cfg["nz"]), (cfg["dx"], cfg["dy"], cfg["dz"]), 4
    boxes, cyls, _ = random_city(*n, *h, lay["seed"], lay["n_boxes"], lay["n_trees"])
    v, t, b, ph = city_meshes(boxes, cyls)
    # algorithmic work: every sample line of every object tile against the
    # object's triangles that are not parallel to the ray
    tests = 0
    for o in range(len(ph)):
        tt = t[b[o]:b[o + 1]]
        used = v[np.unique(tt)]
        lo, hi = used.min(axis=0), used.max(axis=0)
        r = [(max(int(np.floor(lo[a] / h[a])), 0), min(int(np.ceil(hi[a] / h[a])), n[a])) for a in range(3)]
        if any(x0 >= x1 for x0, x1 in r):
            continue
        e1, e2 = v[tt[:, 1]] - v[tt[:, 0]], v[tt[:, 2]] - v[tt[:, 0]]
        live = int(((-e1[:, 1] * e2[:, 2] + e1[:, 2] * e2[:, 1]) != 0).sum())
        tests += (r[1][1] - r[1][0]) * sub * (r[2][1] - r[2][0]) * sub * live
    dev = torch.device("cuda:0")
    vd = torch.as_tensor(v).to(dev)
    td = torch.as_tensor(t).to(dev)
    for _ in range(warmup):
        U.voxelize(n, h, vd, td, b, ph, sub=sub)
    torch.cuda.synchronize()
    cast = []
    w0 = time.perf_counter()
    for _ in range(steps):
        tm = {}
        U.voxelize(n, h, vd, td, b, ph, sub=sub, timing=tm)
        cast.append(tm["cast_ms"])
    torch.cuda.synchronize()
    call_s = (time.perf_counter() - w0) / steps
    k_s = sum(cast) / len(cast) / 1e3
    ncell = n[0] * n[1] * n[2]
    flops = VOX_FLOPS_PER_TEST * tests
    res = {
        "metric": "voxelized cells/s (mesh objects to cell porosity)", "value": ncell / call_s, "unit": "cells/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_call": call_s * 1e3, "higher_is_better": True,
        "dtype": "f64 decisions, f32 porosity", "data": "synthetic seeded city meshes",
        "config": {"workload": "256x256x64 dx=2m city: 40 box buildings (12 triangles), 60 trees "
                               "(16-sided prisms, 64 triangles), 4x4x4 sub-samples per cell",
                   "triangles": int(len(t)), "objects": int(len(ph))},
        "roofline": {"bound": "alu", "kernel": "k_voxelize", "achieved": flops / k_s / 1e12,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": flops / k_s / 1e12 / FP64_PEAK_TFLOPS,
                     "traffic": None, "avg_launch_us": k_s * 1e6, "line_triangle_tests": tests,
                     "flops_per_test": VOX_FLOPS_PER_TEST},
    }
    if with_cpu:
        from oracle.voxelize import voxelize as oracle_voxelize
        c0 = time.perf_counter()
        oracle_voxelize(n, h, v, t, b, ph, sub)
        cs = time.perf_counter() - c0
        res["cpu_baseline"] = {"value": ncell / cs, "unit": "cells/s", "cores": 1, "kind": "oracle",
                               "sample": "the whole 256x256x64 city field (%.1f s), NumPy FP64 per-point rays" % cs}
    print(json.dumps(res), flush=True)


def batch_bench(steps, warmup):
    """The sixteen wind-direction cases (8 directions x 2 variants on uneven
    grids, each on its own stream), the same steps three ways: case after
    case with uf_step; all cases with uf_step_batch (host threads interleave
    the cases' launches); all cases with a uf_batch (one persistent launch
    per stage for every case, the step replayed from two hipGraphs, launch
    shapes from its autotuner).  value is the faster batched path's rate."""
    import torch
    import paper_2204_01117_amd as U
    from uf_layouts import preset, preset_porosity
    p = preset("C3")
    cases = [preset_porosity(p, case=c) for c in range(16)]
    grids = []
    for phi, cfg in cases:
        g = U.Grid(cfg, stream=torch.cuda.Stream())
        g.set_porosity(torch.as_tensor(phi))
        grids.append(g)
    cells = sum(c["nx"] * c["ny"] * c["nz"] for _, c in cases)
    log("C3: %d cases, %d cells in all, shapes %s" % (len(grids), cells,
        sorted({(c["nx"], c["ny"], c["nz"]) for _, c in cases})))
    U.step_batch(grids, warmup)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for g in grids:
        g.step(steps, stats=False)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - w0
    log("sequential uf_step: %.3f ms per step of all cases" % (seq_s / steps * 1e3))
    w0 = time.perf_counter()
    U.step_batch(grids, steps)
    torch.cuda.synchronize()
    thr_s = time.perf_counter() - w0
    log("uf_step_batch: %.3f ms per step of all cases" % (thr_s / steps * 1e3))
    B = U.Batch(grids)
    tune = B.autotune()
    log("autotune", tune)
    B.step(warmup)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    st = B.step(steps)
    torch.cuda.synchronize()
    bat_s = time.perf_counter() - w0
    log("uf_batch: %.3f ms per step of all cases" % (bat_s / steps * 1e3))
    iters = sum(s["cg_iters_total"] for s in st) / (steps * len(grids))
    # value: the faster of the two batched paths, named in config.path
    best_s, path = (bat_s, "uf_batch (one launch per stage for all cases, hipGraphs)") if bat_s <= thr_s else \
        (thr_s, "uf_step_batch (host threads interleave the cases' launches)")
    res = {
        "metric": "cell-updates/s per full RANS step (incl. pressure solve), all cases",
        "value": cells * steps / best_s, "unit": "cell-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": best_s / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic seeded city layouts",
        "config": {"workload": p["workload"] + " (128x128x48, 192x160x48, 256x256x64; 2 m, dt 0.09 s)",
                   "cases": len(grids), "cells": cells, "path": path},
        "sequential_value": cells * steps / seq_s, "step_batch_value": cells * steps / thr_s,
        "uf_batch_value": cells * steps / bat_s, "speedup_vs_sequential": seq_s / best_s,
        "cg_iters_per_step": iters,
        "tuning": {k: {"band": v["band"], "blocks": v["blocks"], "ms": round(v["ms"], 4)} for k, v in tune.items()},
    }
    B.close()
    for g in grids:
        g.close()
    print(json.dumps(res), flush=True)


def gradient_bench(steps, warmup):
    """One full design gradient on the 256x256x64 design case: 21 buildings
    (height and x/y position each) and the trees' porosity, 64 parameters,
    mapped to porosity by smoothed indicators; pedestrian-comfort objective
    at 1.5 m after `steps` steps; forward differences (the paper's method,
    eps = 0.1), i.e. 65 simulations run together through the batched step.
    Beside it the plain single-case step on the same GPU."""
    import numpy as np
    import torch
    import paper_2204_01117_amd as U
    from paper_2204_01117_amd import optimize as O
    from uf_layouts import preset, random_city
    p = preset("C4")
    cfg, lay = dict(p["config"]), p["layout"]
    n, h = (cfg["nx"], cfg["ny"], cfg["nz"]), (cfg["dx"], cfg["dy"], cfg["dz"])
    boxes, cyls, _ = random_city(*n, *h, lay["seed"], lay["n_boxes"], lay["n_trees"])
    design = U.BoxDesign(n, h, [(*b.x, *b.y, *b.z, b.phi) for b in boxes],
                         [(c.cx, c.cy, c.r, *c.z, c.phi) for c in cyls], width=h[0] / 2, dtype="f32")
    g = U.Grid(cfg)
    J = O.SimulationObjective(g, design.porosity, nsteps=warmup, score=lambda gg: gg.plane_objective(1.5))
    theta = design.initial()
    J.many([theta] * (design.nparams + 1))     # builds the pool of grids (warm-up)
    torch.cuda.synchronize()
    J.nsteps = steps
    t0 = time.perf_counter()
    j0, grad = O.forward_difference_gradient(J, theta, 0.1)
    torch.cuda.synchronize()
    grad_s = time.perf_counter() - t0
    g.set_state(J.initial)
    g.set_porosity(design.porosity(theta))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps, stats=False)
    torch.cuda.synchronize()
    single_s = time.perf_counter() - t0
    nsim = design.nparams + 1
    res = {
        "metric": "wall time of one full design gradient (forward differences)", "value": grad_s, "unit": "s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "higher_is_better": False, "dtype": "f32",
        "data": "synthetic seeded city, smoothed building indicators",
        "config": {"workload": "256x256x64 dx=2m, 21 parametrised buildings + 40 trees, 64 parameters, "
                               "plane objective at 1.5 m, %d-step horizon" % steps,
                   "simulations": nsim, "method": "forward differences, eps 0.1, batched"},
        "single_case_ms_per_step": single_s / steps * 1e3,
        "sequential_estimate_s": nsim * single_s, "speedup_vs_sequential": nsim * single_s / grad_s,
        "objective": j0, "gradient_norm": float(np.linalg.norm(grad)),
        "gradient_head": [float(x) for x in grad[:6]], "gradient_tree_porosity": float(grad[-1]),
    }
    J.close()
    g.close()
    print(json.dumps(res), flush=True)


def adjoint_bench(steps, warmup, with_fd=True):
    """One full design gradient on the 256x256x64 design case by the discrete
    adjoint: 21 buildings (height and x/y position each) and the trees'
    porosity, 64 parameters; pedestrian-plane objective ((|u| - 2 m/s)^2 at
    1.5 m plus the stagnation penalty below 0.3 m/s) after `steps` steps of
    the full step (k-omega included) from a state spun up for `warmup`
    steps, with the states checkpointed every 20 steps and each segment
    recomputed in the reverse pass (the timed row).  Beside it: the same
    gradient with every state of the horizon kept in HBM, a plain forward
    run of the horizon, and (unless adjoint_only) the check of the gradient
    in FP64: central differences with h = 1e-3 and 1e-4 on 8 seeded
    parameters (32 simulations batched) against the FP64 adjoint, parameter
    by parameter, with the spread between the two step sizes (large where a
    limiter or clip switches inside the step)."""
    import numpy as np
    import torch
    import paper_2204_01117_amd as U
    from paper_2204_01117_amd import optimize as O
    from uf_layouts import preset, random_city
    p = preset("C4")
    cfg, lay = dict(p["config"]), p["layout"]
    n, h = (cfg["nx"], cfg["ny"], cfg["nz"]), (cfg["dx"], cfg["dy"], cfg["dz"])
    boxes, cyls, _ = random_city(*n, *h, lay["seed"], lay["n_boxes"], lay["n_trees"])
    rows_b = [(*b.x, *b.y, *b.z, b.phi) for b in boxes]
    rows_c = [(c.cx, c.cy, c.r, *c.z, c.phi) for c in cyls]
    design = U.BoxDesign(n, h, rows_b, rows_c, width=h[0] / 2, dtype="f32")
    plane = dict(z_plane=1.5)
    theta = design.initial()
    g = U.Grid(cfg)
    g.set_porosity(design.porosity(theta))
    g.step(warmup, stats=False)
    init = g.state()

    def timed_gradient(checkpoint):
        A = O.AdjointObjective(g, design, [], nsteps=steps, initial_state=init, checkpoint=checkpoint, plane=plane)
        A.value_and_grad(theta)                # allocates the workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J, grad = A.value_and_grad(theta)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, J, grad, A.segment

    adj_s, J, grad, seg = timed_gradient(20)
    hbm_s, J_hbm, grad_hbm, seg_hbm = timed_gradient(None)
    g.set_state(init)
    g.set_porosity(design.porosity(theta))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps, stats=False)
    torch.cuda.synchronize()
    fwd_s = time.perf_counter() - t0
    res = {
        "metric": "wall time of one full design gradient (discrete adjoint)", "value": adj_s, "unit": "s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "higher_is_better": False, "dtype": "f32",
        "data": "synthetic seeded city, smoothed building indicators",
        "config": {"workload": "256x256x64 dx=2m, 21 parametrised buildings + 40 trees, 64 parameters, "
                               "pedestrian plane at 1.5 m, %d-step horizon, full step with k-omega" % steps,
                   "method": "discrete adjoint, checkpoints every %d steps, segments recomputed" % seg},
        "forward_s": fwd_s, "adjoint_over_forward": adj_s / fwd_s,
        "all_states_in_hbm": {"s": hbm_s, "segment": seg_hbm,
                              "max_abs_diff_vs_checkpointed": float(np.abs(grad_hbm - grad).max())},
        "objective": J, "gradient_norm": float(np.linalg.norm(grad)),
        "gradient_head": [float(x) for x in grad[:6]],
    }
    g.close()
    if with_fd:
        cfg64 = dict(cfg, dtype="f64", cg_tol=1e-12, cg_maxit=4000)
        d64 = U.BoxDesign(n, h, rows_b, rows_c, width=h[0] / 2, dtype="f64")
        g64 = U.Grid(cfg64)
        init64 = {f: v.double() for f, v in init.items()}
        A64 = O.AdjointObjective(g64, d64, [], nsteps=steps, initial_state=init64, checkpoint=20, plane=plane)
        t0 = time.perf_counter()
        J64, grad64 = A64.value_and_grad(theta)
        torch.cuda.synchronize()
        adj64_s = time.perf_counter() - t0
        idx = sorted(int(i) for i in np.random.default_rng(4).choice(d64.nparams, 8, replace=False))
        # two step sizes: the limiter, the nu_t cap and the k/omega floors
        # switch somewhere along the design space, so the objective is only
        # piecewise smooth; central differences across such a switch differ
        # from the derivative on either side, and more so the wider the step
        hsteps = (1e-3, 1e-4)
        thetas = []
        for hstep in hsteps:
            for i in idx:
                for sgn in (1.0, -1.0):
                    t = theta.copy()
                    t[i] += sgn * hstep
                    thetas.append(t)
        F = O.SimulationObjective(g64, d64.porosity, nsteps=steps, initial_state=init64,
                                  score=lambda gg: gg.plane_objective(**plane))
        t0 = time.perf_counter()
        vals = F.many(thetas)
        torch.cuda.synchronize()
        fd_s = time.perf_counter() - t0
        nq = len(idx)
        fd = {hs: [(vals[2 * (k * nq + q)] - vals[2 * (k * nq + q) + 1]) / (2 * hs) for q in range(nq)]
              for k, hs in enumerate(hsteps)}
        rel = {hs: [float(abs(grad64[i] - x) / max(abs(x), 1e-300)) for i, x in zip(idx, fd[hs])] for hs in hsteps}
        res["fd_check_fp64"] = {
            "h": list(hsteps), "parameters": idx, "objective": J64, "adjoint_s": adj64_s, "fd_s": fd_s,
            "adjoint": [float(grad64[i]) for i in idx],
            "central_difference": {str(hs): [float(x) for x in fd[hs]] for hs in hsteps},
            "rel_err": {str(hs): rel[hs] for hs in hsteps},
            "rel_err_best_h": [min(rel[hs][q] for hs in hsteps) for q in range(nq)],
            "fd_spread": [float(abs(fd[hsteps[0]][q] - fd[hsteps[1]][q]) / max(abs(fd[hsteps[1]][q]), 1e-300))
                          for q in range(nq)],
            "fp32_adjoint": [float(grad[i]) for i in idx],
            "fp32_rel_err_vs_fp64_adjoint": [float(abs(grad[i] - grad64[i]) / max(abs(grad64[i]), 1e-300))
                                             for i in idx],
        }
        F.close()
        g64.close()
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-probe", action="store_true")
    ap.add_argument("--precond-study", action="store_true")
    ap.add_argument("--voxelize", action="store_true", help="time the mesh voxelizer instead of the step")
    ap.add_argument("--stats-out", default="kernels_512x512x128.md", help="file name under profiles/")
    ap.add_argument("--stats-title", default="Kernel time, 512x512x128 city workload (FP32, multigrid-preconditioned CG)")
    ap.add_argument("--workload", default="C2", choices=["C1", "C2", "slab", "CP", "C3", "C4", "C4A"])
    ap.add_argument("--adjoint-only", action="store_true", help="C4A: skip the forward-difference comparison")
    ap.add_argument("--traffic-summary", metavar="DIR")
    ap.add_argument("--stats-summary", metavar="DIR")
    ap.add_argument("--command", default="", help="the profiling command, recorded in the summary")
    args = ap.parse_args()
    if args.traffic_summary:
        return traffic_summary(args.traffic_summary, args.command, name=args.workload)
    if args.stats_summary:
        return stats_summary(args.stats_summary, args.command, args.stats_out, args.stats_title)
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU; --gpus %d is not supported "
              "(multi-GPU runs would shard independent cases or x-slabs of the grid)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    if args.traffic_probe:
        return traffic_probe(args.workload)
    if args.precond_study:
        return precond_study()
    if args.voxelize:
        return voxelize_bench(args.steps, args.warmup, not args.no_cpu_baseline)
    if args.workload == "C3":
        return batch_bench(args.steps, args.warmup)
    if args.workload == "C4":
        return gradient_bench(args.steps, min(args.warmup, 5))
    if args.workload == "C4A":
        return adjoint_bench(args.steps, args.warmup, not args.adjoint_only)

    p, phi, cfg = workload(args.workload)
    tag = GRID_TAG[args.workload]
    # the oracle's baseline first: its worker processes are forked, which
    # must happen before this process initialises the GPU
    cpu = None
    if not args.no_cpu_baseline and args.workload in ("C1", "C2"):
        cpu = cpu_baseline(args.workload, phi, cfg)
        log("cpu baseline:", json.dumps(cpu))

    import torch
    import paper_2204_01117_amd as U

    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    ncells = nx * ny * nz
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    g = U.Grid(cfg, device="cuda:0")
    g.set_porosity(torch.as_tensor(phi))

    # warm-up, timing every kernel to find the one with the largest share
    g.timer_enable(U.TIMED_KERNELS)
    st = g.step(args.warmup)
    shares = {k: g.timer_read(k)[0] for k in U.TIMED_KERNELS}
    dominant = max((k for k in shares if k in ALG_BYTES_PER_CELL), key=lambda k: shares[k])
    log("warm-up kernel ms:", {k: round(v, 3) for k, v in sorted(shares.items(), key=lambda kv: -kv[1])})

    # timed region: only the dominant kernel is bracketed by events
    g.timer_enable([dominant])
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(stream)
    st = g.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_s = e0.elapsed_time(e1) / 1e3
    secs = max(wall, gpu_s)
    k_ms, k_n = g.timer_read(dominant)
    iters = st["cg_iters_total"]
    alg_bytes = ALG_BYTES_PER_CELL[dominant] * ncells
    avg_s = k_ms / 1e3 / max(k_n, 1)        # over every launch, as rocprof averages
    achieved = alg_bytes / avg_s / 1e9
    result = {
        "metric": "cell-updates/s per full RANS step (incl. pressure solve)",
        "value": ncells * args.steps / secs,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic seeded city layout (porosity field), random-free initial state",
        "config": {"workload": p["workload"], "grid": [nx, ny, nz], "dx_m": cfg["dx"], "dt_s": cfg["dt"],
                   "wind_dir_deg": cfg["wind_dir_deg"], "precond": "multigrid", "cg_tol": cfg["cg_tol"],
                   "turbulence": "k-omega"},
        "cg_iters_per_step": iters / args.steps,
        "cg_iters_max": st.get("cg_iters_max"),
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_for(dominant, tag),
                     "avg_launch_us": avg_s * 1e6, "launches": k_n,
                     "alg_bytes_per_launch": alg_bytes},
        "diagnostics": {"max_div_per_s": st.get("max_div"), "max_cfl": st.get("max_cfl"),
                        "nut_clip_frac": st.get("nut_clip_frac")},
    }
    g.close()
    result["step_hbm"] = step_traffic(iters / args.steps, secs / args.steps * 1e3, ncells, tag)
    result["stream_copy_GBs"] = copy_ceiling_gbs(torch)
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
