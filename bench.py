#!/usr/bin/env python3
"""Throughput of the pseudo-potential LB step with geometric wetting on one MI355X.

Headline workload: the 4096 x 2048 lattice at T = 0.5 T_c (density ratio ~ 725), theta = 45 deg, a wall cap of
radius 400 plus 64 seeded free satellites, FP32 populations stored shifted by the vapour density (f_i - w_i rho_v)
with the EOS evaluated in FP64 below the geometric mean of the coexistence densities, a device check (mass,
non-finite density) every 100 steps. One bench step = one time
step of the whole lattice (density, psi, ghost rows, force, collision, streaming) = one launch of the step kernel.

Prints one JSON line: MLUPS (fluid-node updates per second / 1e6), the HBM-roofline object of the step kernel, the
CPU reference timed on a bounded sample, and side measurements (FP64 on the same lattice, the batched 256-instance
workload against plain per-instance launches).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
# the dominant kernel: the two-step FP32 kernel (two time steps per launch) and the headers it inlines
KERNEL_SRC = [os.path.join(ROOT, "paper_1501_05430_amd", "csrc", n)
              for n in ("lbm_step2.hip", "lbm_device.h", "lbm_internal.h")]
ADJOINT_SRC = [os.path.join(ROOT, "paper_1501_05430_amd", "csrc", n)
               for n in ("lbm_adjoint.hip", "lbm_device.h", "lbm_internal.h")]
STEP1_SRC = [os.path.join(ROOT, "paper_1501_05430_amd", "csrc", n)
             for n in ("lbm_kernels.hip", "lbm_device.h", "lbm_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step2_f32_c3.json")
TRAFFIC_FILE_C4 = os.path.join(ROOT, "profiles", "traffic_step2_f32_batched_c4.json")
TRAFFIC_FILE_MIXED = os.path.join(ROOT, "profiles", "traffic_step2_mixed_c3.json")
TRAFFIC_FILE_ADJ = {"f64": os.path.join(ROOT, "profiles", "traffic_adjoint_f64_c3.json"),
                    "f32": os.path.join(ROOT, "profiles", "traffic_adjoint_f32_c3.json")}
TRAFFIC_FILE_F64 = os.path.join(ROOT, "profiles", "traffic_step2_f64_c3.json")


# HBM-traffic summaries of the step kernels and of the adjoint's fused pass (profiles/traffic_<name>.json), made
# from two rocprofv3 counter runs of this script (FETCH_SIZE, then WRITE_SIZE) by `bench.py --traffic-summary <name>`;
# `run` names the counter runs when two summaries share them, `steps` the time steps per launch (default 2)
TRAFFIC_SPECS = {
    "step2_f32_c3": dict(
        match="k_step2<float, 8, false, false, false>", workload="c3", args="--steps 20 --warmup 5 --no-extras --no-cpu-baseline",
        desc="k_step2<W=8> (two time steps per launch; FP32 storage shifted by rho_v, FP32 arithmetic with the FP64 "
             "EOS in the vapour, tau = 1 BGK, geometric walls), 4096x2048 lattice, T = 0.5 T_c, theta = 45 deg, "
             "65 droplets; default shape"),
    "step2_mixed_c3": dict(
        match="k_step2<float, 4, true, false, false>", workload="c3",
        args="--precision f32_shifted_mixed --steps 20 --warmup 5 --no-extras --no-cpu-baseline",
        desc="k_step2<W=4> in the mixed form (FP32 storage shifted by rho_v and FP32 sums; psi, force, equilibrium "
             "and forcing in FP64), same lattice and shape"),
    "step2_f64_c3": dict(
        match="k_step2<double, 4, false, false, false>", workload="c3", bytes_per_update=144,
        args="--precision f64 --steps 20 --warmup 5 --no-extras --no-cpu-baseline",
        desc="k_step2<double, W=4> (two time steps per launch in FP64: storage and arithmetic), same lattice; "
             "strips of at most 24 output rows"),
    "step2_f32_batched_c4": dict(
        match="k_step2<float, ", exclude=", true", workload="c4", args="--batched-only --steps 40", last=10,
        desc="k_step2 (two time steps per launch, the autotuner's block shape) over the 256-instance batch (sizes "
             "64x32 .. 512x256, T/T_c in [0.6, 0.9], theta in [20, 160] deg, seed 1501), FP32 shifted by rho_v"),
    "step2_general_paper_setting_c3": dict(
        match="k_step2<float, 4, false, true, false>", workload="c3", args="--paper-setting-only --steps 20",
        desc="k_step2<float, W=4, general collision> in the paper's setting (piecewise-linear EOS at a density ratio "
             "of 1000, kappa = 0.5, MRT with diag(0,1,...,1)), same lattice, FP32 shifted by rho_v"),
    "step_f32_c3": dict(
        match="k_step<float, false, true, 8, true, ", workload="c3", steps=1, sources="step",
        args="--steps 20 --warmup 5 --no-extras --no-cpu-baseline --step-variant 8",
        desc="k_step<float, TAU1=true, W=8, PF=true> (one time step per launch, consecutive launches walking the row "
             "strips in alternate directions; FP32 storage shifted by rho_v), 4096x2048 lattice, the headline's "
             "workload with step_variant 8"),
    "adjoint_f64_c3": dict(
        match="ka_fused<false, double>", workload="c3", run="adjoint_c3", args="--adjoint-only", steps=1,
        bytes_per_update=216, state_elem=8, sources="adjoint",
        desc="ka_fused<BGK, FP64 storage> (the adjoint step's fused reverse pass: transposed streaming, collision, "
             "force and psi; f_n and lambda_{n+1} read, lambda_n written), 4096x2048 lattice after 20 steps of the "
             "droplet workload, a seeded random cotangent"),
    "adjoint_f32_c3": dict(
        match="ka_fused<false, float>", workload="c3", run="adjoint_c3", args="--adjoint-only", steps=1,
        bytes_per_update=108, state_elem=4, sources="adjoint",
        desc="ka_fused<BGK, FP32 storage> (lbm_adjoint_step_f32: state and adjoints stored in FP32, FP64 "
             "arithmetic), same lattice and cotangent"),
}
COPY_KERNEL = "k_copy<HIP_vector_type<float, 4u> >"


def traffic_summary(name):
    """profiles/traffic_<name>.json from gpurun_out/prof_<name>_fetch and _write (rocprofv3 --pmc FETCH_SIZE /
    WRITE_SIZE of `bench.py <args>`): the kernel's HBM bytes per launch, each counter scaled by what it reads for
    the float4 copy of known size that the same run performs (bandwidth_ceilings); runs without that copy take the
    scale of the step2_f32_c3 summary."""
    import csv
    from paper_1501_05430_amd import workloads as W
    spec = TRAFFIC_SPECS[name]
    run = spec.get("run", name)
    sources = {"adjoint": ADJOINT_SRC, "step": STEP1_SRC}.get(spec.get("sources"), KERNEL_SRC)
    steps = spec.get("steps", 2)
    runs = {}
    for counter, tag in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        path = os.path.join(ROOT, "gpurun_out", f"prof_{run}_{tag}", "p_counter_collection.csv")
        with open(path) as f:
            rows = [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]
        sel = [r for r in rows
               if spec["match"] in r["Kernel_Name"] and not (spec.get("exclude") and spec["exclude"] in r["Kernel_Name"])]
        if spec.get("last"):
            # the timed launches only: the last ones of the shape the run ended with (an autotuned run first times
            # other shapes, whose traffic differs)
            sel.sort(key=lambda r: int(r["Dispatch_Id"]))
            final = sel[-1]["Kernel_Name"]
            sel = [r for r in sel if r["Kernel_Name"] == final][-spec["last"]:]
        kern = [float(r["Counter_Value"]) for r in sel]
        copy = [float(r["Counter_Value"]) for r in rows if COPY_KERNEL in r["Kernel_Name"]]
        runs[counter] = (sum(kern) / len(kern), len(kern), sum(copy) / len(copy) if copy else None)
    if spec["workload"] == "c3":
        case = W.c3_large()
        nodes = case.fluid_nodes
        pitch = (case.nx + 63) // 64 * 64
        copy_bytes = 4 * 9 * (case.ny - 2) * pitch    # the probe copies an FP32 state of this lattice
        if spec.get("state_elem"):   # the adjoint's arrays: [9][ny-2][nx], unpadded
            state_bytes = spec["state_elem"] * 9 * (case.ny - 2) * case.nx
        else:
            state_bytes = spec.get("bytes_per_update", 72) // 18 * 9 * (case.ny - 2) * pitch   # the kernel's own state
    else:
        nodes = sum(c.fluid_nodes for c in W.c4_batch())
        copy_bytes = state_bytes = None
    if runs["FETCH_SIZE"][2] is not None and copy_bytes:
        calib = {"kernel": f"{COPY_KERNEL} of the bench's bandwidth_ceilings (bw_probe.hip), {copy_bytes:,} bytes "
                           "copied per dispatch",
                 "fetch_kib": round(runs["FETCH_SIZE"][2], 3), "write_kib": round(runs["WRITE_SIZE"][2], 3),
                 "fetch_scale": round(copy_bytes / (1024 * runs["FETCH_SIZE"][2]), 4),
                 "write_scale": round(copy_bytes / (1024 * runs["WRITE_SIZE"][2]), 4)}
    else:
        with open(os.path.join(ROOT, "profiles", "traffic_step2_f32_c3.json")) as f:
            calib = dict(json.load(f)["calibration"])
        calib["kernel"] += " (taken from the step2_f32_c3 run)"
    rd = runs["FETCH_SIZE"][0] * 1024 * calib["fetch_scale"]
    wr = runs["WRITE_SIZE"][0] * 1024 * calib["write_scale"]
    alg = steps * spec.get("bytes_per_update", 72) * nodes
    out = {
        "kernel": spec["desc"],
        "kernel_source_sha256": kernel_sha(sources),
        "kernel_sources": [os.path.relpath(p_, ROOT) for p_ in sources],
        "commands": [f"rocprofv3 --pmc {c} --output-format csv -d gpurun_out/prof_{run}_{t} -o p -- python3 bench.py "
                     f"{spec['args']}" for c, t in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write"))]
                    + [f"python3 bench.py --traffic-summary {name}"],
        "calibration": calib,
        "kernel_counters_kib_per_launch": {"FETCH_SIZE": round(runs["FETCH_SIZE"][0], 1),
                                           "WRITE_SIZE": round(runs["WRITE_SIZE"][0], 1),
                                           "launches_averaged": runs["FETCH_SIZE"][1]},
        "time_steps_per_launch": steps,
        "hbm_read_bytes_per_launch": int(rd),
        "hbm_write_bytes_per_launch": int(wr),
        "hbm_bytes_per_launch": int(rd + wr),
        "algorithmic_bytes_per_launch": alg,
        "traffic_over_algorithmic": round((rd + wr) / alg, 4),
    }
    if state_bytes:
        out["state_bytes"] = state_bytes
    dst = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    with open(dst, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps({"wrote": os.path.relpath(dst, ROOT), "traffic_over_algorithmic": out["traffic_over_algorithmic"]}))


def kernel_sha(sources=None):
    """Hash of a kernel's sources (the step kernel's by default): traffic counters taken from another version are
    not reported."""
    h = hashlib.sha256()
    for path in sources or KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profile_traffic(path, sources=None):
    """(HBM bytes per launch, time steps per launch) from a committed counter summary, if it was taken on the current
    sources of the kernel; (None, 1) otherwise."""
    if not os.path.exists(path):
        return None, 1
    with open(path) as f:
        tr = json.load(f)
    if tr.get("kernel_source_sha256") != kernel_sha(sources):
        return None, 1
    return tr.get("hbm_bytes_per_launch"), tr.get("time_steps_per_launch", 1)


def make_sim(case, precision, check_every=100, **kw):
    import paper_1501_05430_amd as P
    extra = P.fp32_options(case.T_over_Tc, precision, piecewise=kw.get("piecewise"))
    p = P.make_params(case.nx, case.ny, case.T_over_Tc, precision=precision, check_every=check_every, **extra, **kw)
    sim = P.LBM(p)
    sim.apply_wetting(case.theta_bottom, case.theta_top)
    sim.init_droplet(case.xc, case.yc, case.R)
    return sim


def timed_steps(sim, nsteps, inst=0):
    """Device time (ms) of nsteps steps: HIP events that the library records on its own stream right before the
    first queued launch and after the last one (graph replays, device checks included; the closing host
    synchronization excluded). Returns (ms, stable)."""
    import paper_1501_05430_amd as P
    try:
        return sim.step_timed(nsteps, inst=inst), True
    except P.LbmError as e:
        if e.code != 4:
            raise
        return float("nan"), False


def _probe_lib():
    import ctypes as C
    from paper_1501_05430_amd import _build
    lib = C.CDLL(_build.PROBE_LIB)
    lib.bwp_copy.restype = C.c_int
    lib.bwp_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
    lib.bwp_pattern.restype = C.c_int
    lib.bwp_pattern.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p]
    return lib


def bandwidth_ceilings(nx, ny, strip_rows=32, reps=50):
    """What plain memory movement achieves on this GPU, with two buffers of the FP32 step's state size
    (9 x (ny-2) x pitch floats each), ping-pong as the step uses them: a float4 and a float streaming copy (read +
    write bytes), and the step's own access pattern without arithmetic (bw_probe.hip; 72 B per fluid node)."""
    import torch
    lib = _probe_lib()
    pitch = (nx + 63) // 64 * 64
    n = 9 * (ny - 2) * pitch
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    s = torch.cuda.current_stream()
    sp = s.cuda_stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(launch):
        for k in range(4):
            launch(k)
        e0.record(s)
        for k in range(reps):
            launch(k)
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {}
    for vec in (4, 1):
        def cp(k, vec=vec):
            src, dst = (a, b) if k % 2 == 0 else (b, a)
            assert lib.bwp_copy(src.data_ptr(), dst.data_ptr(), 4 * n, vec, sp) == 0
        ms = timed(cp)
        out[f"copy_float{vec if vec > 1 else ''}_gbs"] = round(2 * 4 * n / ms / 1e6, 1)

    def pat(k):
        src, dst = (a, b) if k % 2 == 0 else (b, a)
        assert lib.bwp_pattern(src.data_ptr(), dst.data_ptr(), nx, ny, pitch, strip_rows, k % 2, sp) == 0
    ms = timed(pat)
    out["step_pattern_us"] = round(ms * 1e3, 2)
    out["step_pattern_gbs_alg"] = round(72 * nx * (ny - 2) / ms / 1e6, 1)
    out["buffer_bytes"] = 4 * n
    del a, b
    torch.cuda.empty_cache()
    return out


def cpu_baseline(case, target_s=15.0, max_steps=400):
    """The FP64 reference on the same lattice and initial state, timed on the host's cores. Also returns its state
    (steps taken, fluid-row density, liquid density) for the accuracy report."""
    import oracle
    sim = oracle.Sim(case.nx, case.ny, case.T_over_Tc, theta_bottom=case.theta_bottom, theta_top=case.theta_top)
    sim.init_droplets(case.xc, case.yc, case.R)
    sim.run(2)  # first touch of the population arrays
    n, t0 = 0, time.perf_counter()
    while n < max_steps and time.perf_counter() - t0 < target_s:  # chunks until about target_s of work
        sim.run(5)
        n += 5
    dt = time.perf_counter() - t0
    rho_ref, _ = sim.density()
    ref = (n + 2, rho_ref[1:-1].copy(), sim.coexistence()[1])
    return {
        "value": round(case.fluid_nodes * n / dt / 1e6, 3),
        "unit": "MLUPS",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{case.nx}x{case.ny} lattice (same initial state), FP64 reference, {n} steps after 2 untimed, "
                  f"{dt:.1f} s",
        "single_core": cpu_baseline_one_core(),
    }, ref


def error_vs_oracle(case, ref):
    """The headline configuration (FP32 shifted), the mixed FP32 form and FP64, each stepped on the GPU as far as
    the CPU reference went from the same initial state: max |rho - rho_ref| / rho_l (FP32 forms) and
    / max rho_ref (FP64) over the fluid rows."""
    steps, rho_ref, rho_l = ref
    out = {"steps": steps}
    for precision, scale, key in (("f32_shifted", rho_l, "f32_shifted_max_drho_over_rho_l"),
                                  ("f32_shifted_mixed", rho_l, "f32_shifted_mixed_max_drho_over_rho_l"),
                                  ("f64", np.abs(rho_ref).max(), "f64_max_drho_rel")):
        sim = make_sim(case, precision, check_every=100)
        sim.step(steps)
        rho = sim.rho()[1:-1]
        sim.close()
        out[key] = float(f"{np.abs(rho - rho_ref).max() / scale:.3e}")
    return out


_ONE_CORE = """
import json, sys, time
sys.path.insert(0, sys.argv[1])
import oracle
from paper_1501_05430_amd import workloads as W
case = W.c1_neutral()
sim = oracle.Sim(case.nx, case.ny, case.T_over_Tc, theta_bottom=case.theta_bottom, theta_top=case.theta_top)
sim.init_droplets(case.xc, case.yc, case.R)
sim.run(5)
t0 = time.perf_counter()
n = 0
while time.perf_counter() - t0 < 5.0:
    sim.run(50)
    n += 50
dt = time.perf_counter() - t0
print(json.dumps({"value": round(case.fluid_nodes * n / dt / 1e6, 3), "unit": "MLUPS", "cores": oracle.num_threads(),
                  "sample": f"{case.nx}x{case.ny} lattice, {n} steps, {dt:.1f} s"}))
"""


def cpu_baseline_one_core():
    """The reference on one core (a child process with OMP_NUM_THREADS=1), on the small 200 x 100 lattice."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, "-c", _ONE_CORE, ROOT], env=env, capture_output=True, text=True,
                             timeout=120, check=True).stdout
        return json.loads(out.strip().splitlines()[-1])
    except (subprocess.SubprocessError, ValueError, IndexError) as e:
        return {"error": str(e)[:200]}


def batched_vs_plain(steps_batched=1000, steps_plain=200):
    """256 instances (seeded sizes, angles, temperatures): one launch per step for all of them vs plain launches
    per instance."""
    import paper_1501_05430_amd as P
    from paper_1501_05430_amd import workloads as W
    cases = W.c4_batch()
    params = [P.make_params(c.nx, c.ny, c.T_over_Tc, precision="f32_shifted", check_every=100,
                            **P.fp32_options(c.T_over_Tc, "f32_shifted")) for c in cases]
    nodes = sum(c.fluid_nodes for c in cases)
    batch = P.LBM(params)
    for i, c in enumerate(cases):
        batch.apply_wetting(c.theta_bottom, c.theta_top, inst=i)
        batch.init_droplet(c.xc, c.yc, c.R, inst=i)
    batch.autotune(inst=-1, trial_steps=5)
    batch.step(50, inst=-1)
    ms_b, stable_b = timed_steps(batch, steps_batched, inst=-1)
    batch.close()
    mlups_b = nodes * steps_batched / ms_b / 1e3
    ach = 72 * nodes * steps_batched / ms_b / 1e6
    out = {
        "instances": len(cases), "fluid_nodes": nodes, "dtype": "f32", "precision": "f32_shifted",
        "batched_mlups": round(mlups_b, 1), "batched_stable": stable_b,
        "batched_gbs_alg": round(ach, 1),
        # the batched launches (all instances in each) against the HBM peak: 72 B per fluid node and step
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": profile_traffic(TRAFFIC_FILE_C4)[0],
                     "launch": "k_step2 (two time steps per launch, every instance in each)"},
    }
    if steps_plain <= 0:
        return out
    # plain per-instance launches (each instance its own context and graph), same total work per step
    sims = []
    for c, p in zip(cases, params):
        s = P.LBM(p)
        s.apply_wetting(c.theta_bottom, c.theta_top)
        s.init_droplet(c.xc, c.yc, c.R)
        sims.append(s)
    import torch
    for s in sims:
        s.step(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.step(steps_plain)
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t0
    for s in sims:
        s.close()
    mlups_p = nodes * steps_plain / dt_plain / 1e6
    out["plain_sequential_mlups"] = round(mlups_p, 1)
    out["speedup"] = round(mlups_b / mlups_p, 2)
    return out


def adjoint_rate(case, calls=30, dtype="f64", **kw):
    """lbm_adjoint_step on the same lattice (FP64 state, a seeded random cotangent): time per reverse step. Its
    unavoidable traffic is 216 B per node (108 with dtype="f32"): f_n and lambda_{n+1} read, lambda_n written. kw:
    further lattice options (EOS, collision, kappa)."""
    import torch
    sim = make_sim(case, "f64", check_every=0, enable_adjoint=True, **kw)
    sim.step(20)
    f = sim.populations(device=True)
    if dtype == "f32":  # lbm_adjoint_step_f32: FP32 state and adjoints (FP64 arithmetic)
        f = f.float()
    g = torch.Generator(device=f.device)
    g.manual_seed(1501)
    lam1 = torch.randn(f.shape, generator=g, device=f.device, dtype=f.dtype)
    lam0 = torch.empty_like(lam1)
    theta_bar = torch.zeros((2, case.nx), dtype=torch.float64, device=f.device)
    G_bar = torch.zeros(2, dtype=torch.float64, device=f.device)
    sim.adjoint_step(f, lam1, lam0, theta_bar, G_bar)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    with torch.cuda.stream(sim.stream):  # queued back to back on the library's stream, as a reverse rollout runs them
        for _ in range(calls):
            sim.adjoint_step(f, lam1, lam0, theta_bar, G_bar)
    e1.record(sim.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / calls
    finite = bool(torch.isfinite(lam0).all().item())
    sim.close()
    nbytes = 216 if dtype == "f64" else 108
    out = {"ms_per_step": round(ms, 4), "mlups": round(case.fluid_nodes / ms / 1e3, 1),
           "gbs_alg": round(nbytes * case.fluid_nodes / ms / 1e6, 1), "finite": finite}
    if not kw and case.nx == 4096 and case.ny == 2048:
        # the fused pass's measured HBM bytes per launch (committed counter summary of this lattice), if current
        out["fused_pass_traffic"] = profile_traffic(TRAFFIC_FILE_ADJ[dtype], ADJOINT_SRC)[0]
    return out


def piecewise_rate(case, steps=2000, kappa=0.0):
    """The same lattice and droplets with the piecewise-linear EOS of Eq. 11 at a density ratio of 1000 (Table 1:
    theta = 0.2, -0.01, 0.33333 with rho_v = 1), FP32 shifted by rho_v as the headline run. kappa != 0 adds the
    surface-tension source of Eq. 16-17 with the relaxation matrix diag(0,1,...,1) of Sec. 3.1 (the MRT collision,
    in the general instance of the two-step kernel): the paper's own setting."""
    pw = (0.2, -0.01, 0.33333, 1.0, 1000.0)
    sim = make_sim(case, "f32_shifted", check_every=100, piecewise=pw, kappa=kappa)
    sim.step(50)
    m0 = sim.mass()
    ms, stable = timed_steps(sim, steps)
    d = sim.diag()
    m1 = sim.mass()
    sim.close()
    nodes = case.fluid_nodes
    ach = 72 * nodes * steps / ms / 1e6
    return {"mlups": round(nodes * steps / ms / 1e3, 1), "gbs_alg": round(ach, 1),
            "frac_of_hbm_peak": round(ach / PEAK_HBM_GBS, 4), "steps": steps,
            "stable": stable and d["nonfinite"] == 0, "psi_clamps": d["psi_clamps"], "mass_drift": abs(m1 - m0) / m0}


def martys_chen_rate(case, steps=1000):
    """The comparison method of Sec. 3 on the same lattice and droplets: Martys-Chen walls (the fluid-solid force of
    Eq. 14, G_w = -1.6 on both walls, about 94 deg in Sec. 3.1's setting) with the piecewise-linear EOS of Table 1
    at a density ratio of 10 and kappa = 0.5, FP32 shifted by rho_v, through the general instance of the two-step
    kernel."""
    pw = (0.25, -0.02, 0.3, 1.0, 10.0)
    sim = make_sim(case, "f32_shifted", check_every=100, piecewise=pw, kappa=0.5, boundary="martys_chen",
                   G_w=(-1.6, -1.6))
    sim.step(50)
    ms, stable = timed_steps(sim, steps)
    d = sim.diag()
    sim.close()
    nodes = case.fluid_nodes
    ach = 72 * nodes * steps / ms / 1e6
    return {"mlups": round(nodes * steps / ms / 1e3, 1), "gbs_alg": round(ach, 1),
            "frac_of_hbm_peak": round(ach / PEAK_HBM_GBS, 4), "steps": steps,
            "stable": stable and d["nonfinite"] == 0}


def mixed_rate(case, steps=1000):
    """The FP32 storage form with the force and equilibrium in FP64 (LBM_F32_SHIFTED_MIXED) on the same lattice,
    in the same launch configuration: the same 72 B per fluid node and step."""
    sim = make_sim(case, "f32_shifted_mixed", check_every=100)
    sim.step(50)
    ms, stable = timed_steps(sim, steps)
    d = sim.diag()
    sim.close()
    nodes = case.fluid_nodes
    ach = 72 * nodes * steps / ms / 1e6
    return {"mlups": round(nodes * steps / ms / 1e3, 1), "gbs_alg": round(ach, 1),
            "frac_of_hbm_peak": round(ach / PEAK_HBM_GBS, 4), "steps": steps,
            "stable": stable and d["nonfinite"] == 0}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the step kernel's block shape first (default: the library's defaults)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the 256-instance batched leg and print its JSON (for profiling that launch)")
    ap.add_argument("--paper-setting-only", action="store_true",
                    help="only the paper's setting on the headline lattice (piecewise EOS, kappa = 0.5, MRT), --steps")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint legs on the headline lattice and print their JSON (for profiling)")
    ap.add_argument("--step-variant", type=int, default=0,
                    help="force the headline's step shape (lbm_params.step_variant: 1..8 one-step kernel, 9..12 "
                         "two-step; 0 = library default), to profile a kernel the default does not run")
    ap.add_argument("--precision", default="f32_shifted", choices=["f32_shifted", "f32_shifted_mixed", "f64"],
                    help="the timed form: FP32 arithmetic (default), the mixed form (FP64 force and equilibrium) "
                         "or FP64")
    ap.add_argument("--traffic-summary", metavar="NAME", choices=sorted(TRAFFIC_SPECS),
                    help="write profiles/traffic_NAME.json from the two counter runs under gpurun_out/ and exit")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(args.traffic_summary)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs each lattice on a single MI355X, with no "
              f"collectives (asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1501_05430_amd as P
    from paper_1501_05430_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    P.load()

    if args.batched_only:
        print(json.dumps({"batched_256": batched_vs_plain(steps_batched=args.steps, steps_plain=0)}), flush=True)
        return
    if args.paper_setting_only:
        print(json.dumps({"paper_setting_ratio1000_kappa05_same_lattice":
                          piecewise_rate(W.c3_large(), steps=args.steps, kappa=0.5)}), flush=True)
        return
    if args.adjoint_only:
        case = W.c3_large()
        print(json.dumps({"adjoint_fp64_same_lattice": adjoint_rate(case),
                          "adjoint_fp32_storage_same_lattice": adjoint_rate(case, dtype="f32")}), flush=True)
        return

    case = W.c3_large()
    ceilings = bandwidth_ceilings(case.nx, case.ny)
    sim = make_sim(case, args.precision, check_every=100,
                   **({"step_variant": args.step_variant} if args.step_variant else {}))
    if args.autotune:
        sim.autotune(trial_steps=10)
    sim.step(args.warmup)
    ms, stable = timed_steps(sim, args.steps)
    diag = sim.diag()
    theta = sim.measure_contact_angle((1700, 2400, 1, 200), wall=0)
    waves2 = sim.tuning()["waves2"]  # wavefronts per block of the two-step kernel the run used
    sim.close()
    nodes = case.fluid_nodes
    ms_step = ms / args.steps
    mlups = nodes * args.steps / ms / 1e3
    bytes_alg = 72 * nodes  # 9 FP32 populations read + 9 written per fluid node and step
    achieved = bytes_alg / (ms_step * 1e-3) / 1e9

    mixed = args.precision == "f32_shifted_mixed"
    f64 = args.precision == "f64"
    if f64:
        bytes_alg = 144 * nodes  # 9 FP64 populations read + 9 written per fluid node and step
        achieved = bytes_alg / (ms_step * 1e-3) / 1e9
    traffic, per_launch = profile_traffic(TRAFFIC_FILE_F64 if f64 else (TRAFFIC_FILE_MIXED if mixed else TRAFFIC_FILE))
    if args.step_variant:  # a forced shape: the committed counters are the default kernel's
        traffic, per_launch = None, 1

    out = {
        "metric": "MLUPS & % HBM roofline; FP32/batched/adjoint vs plain FP64 at stated error",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if f64 else ("f32+f64" if mixed else "f32"),
        "data": "synthetic",
        "config": {
            "workload": case.name, "nx": case.nx, "ny": case.ny, "fluid_nodes": nodes, "T_over_Tc": 0.5,
            "theta_deg": 45, "droplets": len(case.xc), "seed": W.SEED, "precision": ("f64" if f64 else
                                                          "f32_shifted_mixed (rho0 = rho_v; FP32 storage and sums, FP64 "
                                                          "psi, force and equilibrium)" if mixed else
                                                          "f32_shifted (rho0 = rho_v; FP64 EOS in vapour)"),
            "check_every": 100, "stable": stable, "mass_at_last_check": diag["mass"],
            "measured_theta_deg": round(math.degrees(theta[0]), 3),
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            # the dominant kernel: two time steps per launch; traffic is its HBM bytes per launch (counters, when
            # current), traffic_gbs those bytes over this run's time per launch
            "kernel": (f"the shape step_variant {args.step_variant} selects" if args.step_variant else
                       f"k_step2<{'double' if f64 else 'float'}, {waves2}, {'true' if mixed else 'false'}, false, "
                       "false> (two time steps per launch; one launch in 50 its checked instance)"),
            "steps_per_launch": 1 if 0 < args.step_variant <= 8 else 2,
            "traffic_gbs": round(traffic / (per_launch * ms_step * 1e-3) / 1e9, 1) if traffic else None,
            # plain memory movement on this GPU (bw_probe.hip): float4 / float ping-pong copies of the state's size
            # and the step's access pattern without arithmetic
            "copy_gbs_on_this_gpu": ceilings["copy_float4_gbs"],
            "ceilings": ceilings,
        },
    }

    if not args.no_extras:
        sim64 = make_sim(case, "f64", check_every=100)
        sim64.step(50)
        ms64, st64 = timed_steps(sim64, 1000)
        sim64.close()
        out["extras"] = {
            "fp64_same_lattice": {"mlups": round(nodes * 1000 / ms64 / 1e3, 1),
                                  "gbs_alg": round(144 * nodes * 1000 / ms64 / 1e6, 1),
                                  "frac_of_hbm_peak": round(144 * nodes * 1000 / ms64 / 1e6 / PEAK_HBM_GBS, 4),
                                  "stable": st64},
            "f32_shifted_mixed_same_lattice": mixed_rate(case),
            "batched_256": batched_vs_plain(),
            "adjoint_fp64_same_lattice": adjoint_rate(case),
            "adjoint_fp32_storage_same_lattice": adjoint_rate(case, dtype="f32"),
            "piecewise_eos_ratio1000_same_lattice": piecewise_rate(case),
            "paper_setting_ratio1000_kappa05_same_lattice": piecewise_rate(case, kappa=0.5),
            "martys_chen_ratio10_kappa05_same_lattice": martys_chen_rate(case),
            # the reverse step in the paper's setting (MRT form with the surface-tension source)
            "adjoint_paper_setting_same_lattice": adjoint_rate(case, piecewise=(0.2, -0.01, 0.33333, 1.0, 1000.0),
                                                               kappa=0.5),
        }
        out["extras"]["adjoint_fp64_same_lattice"]["vs_forward_fp64"] = round(
            out["extras"]["adjoint_fp64_same_lattice"]["mlups"] / out["extras"]["fp64_same_lattice"]["mlups"], 3)

    if not args.no_cpu_baseline:
        out["cpu_baseline"], ref = cpu_baseline(case)
        out["error_vs_oracle"] = error_vs_oracle(case, ref)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
