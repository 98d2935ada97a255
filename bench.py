"""Throughput of the fused D2Q9 step on one MI355X.

Workload (default): the 4096 x 1024 channel with a cylinder of D = 80 at
x = 10 D, MRT collision, populations stored as FP32 offsets f - w, Zou & He
velocity inlet and pressure outlet, bounce-back walls, Re = 200, seeded
velocity noise 1e-4.  One step = one pass of the whole hot path: pull
streaming with half-way bounce-back, inlet and outlet columns, collision,
momentum-exchange force and mass reduction.  The same lattice is then timed
with the neural outflow active (MLP 27-64-64-3 fused into the step).

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]

Counter figures for roofline.traffic are taken with rocprofv3 (see
profiles/step_kernel_<nx>x<ny>_traffic.txt for the commands): the HBM
counters FETCH_SIZE and WRITE_SIZE of the step kernel, each scaled by what
the same counter reads for a plain copy of known size (``--calibration-copy``).
``--write-traffic`` turns those CSV files into that summary (for the lattice
size given by --nx/--ny), stamped with a hash of the kernel sources; traffic
is reported only while the hash matches.
"""
import argparse
import csv
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_NODE = {"fp64": 144, "fp32": 72, "fp16": 36}   # 9 loads + 9 stores
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2506_05293_amd", "csrc")
RESULTS = os.path.join(ROOT, "results")
# the Zou & He step runs two lattice steps per launch of this kernel
STEP_KERNEL, STEPS_PER_LAUNCH = "k_step3<", 3
CALIB_BYTES = 151 * 1024 * 1024     # bytes read (and written) by the calibration copy


STEP_SOURCES = ("d2q9_dev.hpp", "lbm_internal.hpp", "node_dev.hpp", "mlp_dev.hpp",
                "lbm_kernels.hip", "lbm_api.cpp")


def kernel_source_hash():
    """Hash of the sources the step kernel and its launcher are built from."""
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def calibration_copy():
    """A plain device copy of CALIB_BYTES (torch copy_), five dispatches."""
    import torch
    a = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print("calibration copy done", flush=True)


def _median_counter(path, name_part):
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if name_part in r["Kernel_Name"]]
    if not vals:
        raise SystemExit(f"no dispatch of {name_part!r} in {path}")
    return statistics.median(vals)


def traffic_file(nx, ny):
    return os.path.join(ROOT, "profiles", f"step_kernel_{nx}x{ny}_traffic.txt")


def write_traffic(nx, ny, step_fetch, step_write, copy_fetch, copy_write, command_note):
    """Scale the step kernel's FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by
    the copy's reading of CALIB_BYTES and store bytes per launch."""
    kib = CALIB_BYTES / 1024.0
    f_scale = kib / _median_counter(copy_fetch, "copyBuffer")
    w_scale = kib / _median_counter(copy_write, "copyBuffer")
    fetch = _median_counter(step_fetch, STEP_KERNEL) * f_scale * 1024
    write = _median_counter(step_write, STEP_KERNEL) * w_scale * 1024
    lines = [f"source_hash={kernel_source_hash()}",
             f"kernel={STEP_KERNEL}", f"steps_per_launch={STEPS_PER_LAUNCH}",
             f"fetch_bytes_per_launch={fetch:.0f}",
             f"write_bytes_per_launch={write:.0f}",
             f"fetch_scale={f_scale:.4f}", f"write_scale={w_scale:.4f}",
             f"commands={command_note}"]
    with open(traffic_file(nx, ny), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def stored_traffic(nx, ny):
    """HBM bytes per lattice step of the FP32 nx x ny lattice from its
    counter summary (a launch of the step kernel advances STEPS_PER_LAUNCH
    steps), or None when there is none or the kernel sources changed since
    the counters were taken."""
    path = traffic_file(nx, ny)
    if not os.path.exists(path):
        return None
    kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l)
    if kv.get("source_hash") != kernel_source_hash() or kv.get("kernel") != STEP_KERNEL:
        return None
    per_launch = float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    return per_launch / int(kv["steps_per_launch"])


def step_roofline(nodes, ms_per_step, spl, precision, traffic_per_step):
    """The roofline object of the step: algorithmic bytes per launch (72 B
    per node and step at FP32 times the node-steps of one launch) over the
    launch's mean duration; the counter traffic (bytes per step) beside it."""
    bpn = BYTES_PER_NODE[precision]
    launch_ms = ms_per_step * spl
    gbs = bpn * nodes * spl / (launch_ms * 1e-3) / 1e9
    tr = None if traffic_per_step is None else traffic_per_step / (ms_per_step * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": tr,
            "traffic_frac": None if tr is None else tr / HBM_PEAK_GBS,
            "bytes_per_node_step": bpn, "steps_per_launch": spl,
            "algorithmic_bytes_per_launch": bpn * nodes * spl, "launch_ms": launch_ms,
            # a launch of spl steps needs to move the populations only once:
            # its own minimum is bpn / spl per node-step
            "launch_minimum_bytes_per_node_step": bpn / spl,
            "launch_minimum_frac": gbs / spl / HBM_PEAK_GBS,
            "kernel": {3: "k_step3 (three fused pull stream-collide steps per launch)",
                       2: "k_step2 (two fused pull stream-collide steps per launch)"}.get(
                           spl, "k_step (fused pull stream-collide)")}


def c2_case(nx, ny):
    from paper_2506_05293_amd import geometry
    D = 80.0 * nx / 4096
    mask = geometry.cylinder(nx, ny, 10 * D, ny // 2, D)
    return mask, 3 * 0.05 * D / 200 + 0.5


def random_mlp(seed=0):
    """Random-initialised 27-64-64-3 network (Glorot-uniform scale) with
    standardisation maps of the size of FP32 population offsets."""
    rng = np.random.default_rng(seed)

    def glorot(o, i):
        a = np.sqrt(6.0 / (o + i))
        return rng.uniform(-a, a, (o, i))
    return {"w1": glorot(64, 27), "b1": np.zeros(64), "w2": glorot(64, 64), "b2": np.zeros(64),
            "w3": 0.01 * glorot(3, 64), "b3": np.zeros(3),
            "mu_in": np.zeros(27), "sd_in": np.full(27, 0.01),
            "mu_out": np.zeros(3), "sd_out": np.full(3, 1e-4)}


def time_steps(lat, steps, warmup, torch):
    lat.step(warmup)
    lat.sync()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps     # ms per step (one step kernel each)


# Algorithmic HBM bytes per node and segment step of the CBC trainer (FP32):
# forward 9 pulled reads + 9 writes; backward (streaming and collision
# adjoints fused) 9 gathered adjoint reads + 9 pulled state reads + 9 writes.
CBC_TRAIN_BYTES_PER_NODE_STEP = 4 * (18 + 27)


def time_cbc_training(torch, steps=20, warmup=3):
    """Adam steps of the closed-loop CBC trainer on the shape of the
    paper's training set: 110 start states for each of n_t = 5, 10, 25 on
    the 200 x 400 convected-vortex lattice (strips of 53 columns), FP32.
    The start states are the vortex's initial state placed at the outlet
    (the cost does not depend on the values)."""
    from paper_2506_05293_amd import lbm, workloads
    case = workloads.convected_vortex(nx=200, ny=400, x0=185.0)
    ny, w, n_ts = 400, 53, [5] * 110 + [10] * 110 + [25] * 110
    lat = lbm.Lattice(case["mask"], case["tau"], precision="fp32", collision="bgk",
                      lateral="periodic", u_in=case["u0"], noise_amp=0.0)
    lat.init_fields(case["rho"], case["ux"], case["uy"])
    strip = lat.populations()[:, :, -w:]
    del lat
    a0 = np.ascontiguousarray(np.broadcast_to(strip, (len(n_ts),) + strip.shape))
    ref = np.zeros((len(n_ts), 3, ny, 25))
    ref[:, 0] = 1.0
    ref[:, 1] = case["u0"]
    rng = np.random.default_rng(0)
    net = {"w1": rng.standard_normal((20, 9)) * 0.47, "b1": np.zeros(20),
           "w2": rng.standard_normal((20, 20)) * 0.32, "b2": np.zeros(20),
           "w3": rng.standard_normal((2, 20)) * 0.02, "b3": np.zeros(2),
           "mu_in": np.zeros(9), "sd_in": np.full(9, 1e-3), "leaky_slope": 0.01,
           "sigma_scale": 1.0, "sigma_shift": 0.0, "kappa_scale": 1.0, "kappa_shift": 0.0}
    tr = lbm.CbcTrainer(a0, ref, np.array(n_ts, np.int32), net, tau=case["tau"],
                        mach=case["ma"], length=200.0, precision="fp32", eps=1e-16)
    tr.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    tr.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    node_steps = sum(n_ts) * ny * w
    gbs = CBC_TRAIN_BYTES_PER_NODE_STEP * node_steps / (ms * 1e-3) / 1e9
    return {"ms_per_adam_step": ms, "segments": len(n_ts), "segment_steps": sum(n_ts),
            "node_steps_per_s": node_steps / (ms * 1e-3),
            "algorithmic_GBps": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
            "bytes_per_node_step": CBC_TRAIN_BYTES_PER_NODE_STEP,
            "setting": "110 starts x n_t in {5, 10, 25}, 200x400 vortex lattice, strips of 53 "
                       "columns, FP32, forward + adjoint + Adam"}


# Algorithmic HBM bytes per node and step of the D3Q19 step (FP32 offsets):
# 19 pulled reads + 19 writes.
D3Q19_BYTES_PER_NODE = 4 * 38


def time_d3q19(torch, steps=500, warmup=50, nx=256, ny=128, nz=128):
    """The D3Q19 step on a walled channel nx x ny x nz with a sphere of
    diameter ny/4 at x = nx/4, FP32 offsets, Re = 100 (u_in 0.05)."""
    from paper_2506_05293_amd import lbm
    d = ny / 4
    Z, Y, X = np.mgrid[0:nz, 0:ny, 0:nx]
    mask = (((X - nx / 4) ** 2 + (Y - (ny - 1) / 2) ** 2 + (Z - (nz - 1) / 2) ** 2)
            <= (d / 2) ** 2).astype(np.uint8)
    tau = 0.5 + 3 * 0.05 * d / 100
    lat = lbm.Lattice3D(mask, tau, precision="fp32", lateral="walls", u_in=0.05,
                        history_cap=steps + warmup)
    lat.step(warmup)
    lat.sync()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    fo = lat.forces()
    assert fo.nonfinite == 0
    nodes = nx * ny * nz
    gbs = D3Q19_BYTES_PER_NODE * nodes / (ms * 1e-3) / 1e9
    return {"mlups": nodes / (ms * 1e-3) / 1e6, "ms_per_step": ms,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "bytes_per_node": D3Q19_BYTES_PER_NODE,
                         "kernel": "k3_step (force sums reduced every 16 steps by k3_reduce)"},
            "drag_fx_last": fo.fx,
            "setting": f"D3Q19 BGK {nx}x{ny}x{nz} walled channel, sphere D={d:g} at x={nx // 4}, "
                       "FP32 offsets, Zou-He faces, Re=100"}


def time_batch(torch, steps=1000, warmup=200, n_pairs=64, launch="per_step"):
    """The training-data batch: n_pairs cylinder pairs (128 lattices, 33.4M
    nodes at 64 pairs), MRT with the study rates, FP32, one launch per step."""
    from paper_2506_05293_amd import lbm, workloads
    lattices, _, rows = workloads.training_pairs(n_pairs, 3)
    nodes = sum(L["mask"].size for L in lattices)
    b = lbm.Batch(lattices, collision="mrt", lateral="periodic", noise_amp=1e-4, history_cap=0,
                  log_rows=rows, s_e=1.0, s_eps=1.0, s_q=1.0, launch=launch)
    b.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    assert not np.any(b.retired())
    gbs = 72 * nodes / (ms * 1e-3) / 1e9
    return {"mlups": nodes / (ms * 1e-3) / 1e6, "ms_per_step": ms, "nodes": int(nodes),
            "lattices": len(lattices),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "bytes_per_node": 72,
                         "kernel": "k_batch_step (one launch per step)"},
            "setting": f"{n_pairs} cylinder pairs (D 20-40, Re 40-400), MRT s=1, FP32 offsets, "
                       f"launch {launch}"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_worker(args):
    """One process: the FP64 oracle on its own copy of the lattice for
    ~`seconds` (single thread); returns (node updates, seconds)."""
    nx, ny, seconds = args
    from threadpoolctl import threadpool_limits
    from oracle.solver import Lattice as Oracle
    mask, tau = c2_case(nx, ny)
    with threadpool_limits(limits=1):
        o = Oracle(mask, tau, collision="mrt", lateral="walls", u_in=0.05, noise_amp=1e-4, seed=2)
        t0 = time.perf_counter()
        n = 0
        while n == 0 or time.perf_counter() - t0 < seconds:
            o.step(1)
            n += 1
        return nx * ny * n, time.perf_counter() - t0


def cpu_baseline(nx, ny, seconds=15.0, all_cores=True):
    """The FP64 oracle (single thread) on the same lattice for as many whole
    steps as fit in ~`seconds` (at least one); then, optionally, one oracle
    process per core of this process's CPU set (at most 16), each on its own
    copy of a quarter-height lattice, for the aggregate figure."""
    nodes, dt = _oracle_worker((nx, ny, seconds))
    out = {"value": nodes / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
           "cpu": cpu_model(),
           "sample": f"{nodes // (nx * ny)} steps of the same {nx}x{ny} MRT lattice, FP64 NumPy, "
                     "1 thread"}
    if all_cores:
        import multiprocessing as mp
        procs = max(1, min(16, len(os.sched_getaffinity(0))))
        sub = max(64, ny // 4)
        ctx = mp.get_context("spawn")
        with ctx.Pool(procs) as pool:
            res = pool.map(_oracle_worker, [(nx, sub, 10.0)] * procs)
        out["all_cores"] = {"value": sum(n / t for n, t in res) / 1e6, "unit": "MLUPS",
                            "cores": procs,
                            "sample": f"{procs} processes, each the oracle on its own {nx}x{sub} "
                                      "copy of the lattice for ~10 s, 1 thread each"}
    return out


def _jsonable(o):
    if isinstance(o, dict):
        return {str(k): _jsonable(v) for k, v in o.items()
                if not hasattr(v, "data_ptr") and k not in ("batch",)}
    if isinstance(o, (list, tuple)):
        return [_jsonable(v) for v in o]
    if isinstance(o, np.ndarray):
        return o.tolist()
    if isinstance(o, (np.floating, np.integer)):
        return o.item()
    return o


def _progress(name, res):
    keys = ("cd_mean", "cl_rms", "st", "mlups", "fallback_per_step", "nonfinite")
    print(json.dumps({"case": name, **{k: res.get(k) for k in keys}}), flush=True)


def train_study(scale):
    """Training data (one batched launch per 2000 steps) and Adam training of
    every network shape of experiments.NETWORKS; writes
    results/network_<name>.json and results/training.json and returns the
    networks."""
    import torch
    from paper_2506_05293_amd import experiments
    n = lambda k: max(1, int(k * scale))
    data = experiments.generate_data(steps=n(80_000), log_every=32, progress=_progress)
    idx = experiments.select_rows(data)
    x, t = data["x"][idx].contiguous(), data["t"][idx].contiguous()
    gen = {k: data[k] for k in ("wall_s", "nodes", "mlups", "slots", "rows_per_slot")}
    gen.update(samples=int(x.shape[0]), retired_lattices=int(data["retired"].sum()),
               pairs=len(data["pairs"]))
    print(json.dumps({"generate": gen}), flush=True)
    del data
    torch.cuda.empty_cache()
    nets, log = {}, {}
    for name, (n_in, hidden) in experiments.NETWORKS.items():
        tr = experiments.train_network(x, t, n_in=n_in, hidden=hidden, steps=n(20_000))
        print(json.dumps({"train": name, "loss_curve": tr["loss_curve"][-3:],
                          "wall_s": tr["wall_s"]}), flush=True)
        nets[name] = {k: np.asarray(v, np.float64) for k, v in tr["weights"].items()}
        with open(os.path.join(RESULTS, f"network_{name}.json"), "w") as f:
            json.dump(_jsonable(tr["weights"]), f)
        log[name] = _jsonable({k: v for k, v in tr.items() if k != "weights"})
    with open(os.path.join(RESULTS, "training.json"), "w") as f:
        json.dump({"generate": gen, "train": log}, f, indent=1)
    return nets


def _suffix(mass_bound):
    return "" if mass_bound == 1e-2 else f"_bound{mass_bound:g}"


def load_networks():
    from paper_2506_05293_amd import experiments
    nets = {}
    for name in experiments.NETWORKS:
        path = os.path.join(RESULTS, f"network_{name}.json")
        if not os.path.exists(path):
            return None
        with open(path) as f:
            nets[name] = {k: np.asarray(v, np.float64) for k, v in json.load(f).items()}
    return nets


def run_studies(which, scale, nn_switch=0, mass_bound=1e-2, study_seeds=(2,)):
    """train: training data and training.  nn: truncated-domain outflow study.
    naca: NACA0012 study.  all: the three in turn.  nn and naca reuse the
    networks in results/ when they exist (else they train first)."""
    from paper_2506_05293_amd import experiments
    os.makedirs(RESULTS, exist_ok=True)
    n = lambda k: max(1, int(k * scale))
    cbc_runs = {"cbc_train": ("cbc_training.json", {}),
                # two Mach numbers in one training set, Ma 0.2 between them held out
                "cbc_train_mach": ("cbc_training_mach.json", dict(
                    flows=[{}, {"ma": 0.1}],
                    holdout={"ma0.2": dict(ma=0.2), "ma0.15": dict(ma=0.15),
                             "ma0.25": dict(ma=0.25),
                             "strong_ma0.2": dict(ma=0.2, beta=0.8, rc=25.0, x0=140.0)}))}
    for name, (out, kw) in cbc_runs.items():
        if which not in (name, "all"):
            continue
        res = experiments.cbc_training_study(adam_steps=n(2000), progress=_progress, **kw)
        with open(os.path.join(RESULTS, out), "w") as f:
            json.dump(_jsonable(res), f, indent=1)
        print(json.dumps({name: {
            "loss_before": res["loss_before"], "loss_after": res["loss_after"],
            "ms_per_adam_step": res["ms_per_adam_step"], "loss_per_flow": res["loss_per_flow"],
            "vortex": {k: {a: r[a] for a in ("max", "final", "mean", "finite")}
                       for k, r in res["vortex"]["runs"].items()},
            **{part: {h: {k: r["mean"] for k, r in v["runs"].items()}
                      for h, v in res[part].items()} for part in ("trained_flows", "held_out")}}}),
              flush=True)
    if which in ("cbc_train", "cbc_train_mach"):
        return
    if which in ("vortex", "all"):
        res = experiments.vortex_study(steps=max(10, n(600) // 10 * 10), progress=_progress)
        with open(os.path.join(RESULTS, "vortex_study.json"), "w") as f:
            json.dump(_jsonable(res), f, indent=1)
        print(json.dumps({"vortex": {k: {a: r[a] for a in ("max", "final", "mean", "finite")}
                                     for k, r in res["runs"].items()}}), flush=True)
        if which == "vortex":
            return
    nets = None if which in ("train", "all") else load_networks()
    if nets is None:
        nets = train_study(scale)
    if which in ("nn_train", "all"):
        res = experiments.nn_rollout_training_study(
            nets["paper_9x20"], adam_steps=n(5000), eval_steps=n(150_000),
            eval_seeds=study_seeds, progress=_progress)
        with open(os.path.join(RESULTS, "nn_rollout_training.json"), "w") as f:
            json.dump(_jsonable(res), f, indent=1)
        print(json.dumps({"nn_train": _jsonable({
            k: res[k] for k in ("loss_before", "loss_after", "val_loss_before", "val_loss_after",
                                "zou_he_loss", "zou_he_val_loss", "ms_per_adam_step")}),
            "nn_train_rel_err_mean": _jsonable({re: r["rel_err_mean"]
                                                for re, r in res["evaluation"].items()})}),
            flush=True)
        if which == "nn_train":
            return
    if which in ("nn_drift", "all"):
        with open(os.path.join(RESULTS, "nn_rollout_training.json")) as f:
            trained = {k: np.asarray(v, np.float64) for k, v in json.load(f)["network"].items()}
        res = experiments.drift_trace({
            "rollout_m0.01": (trained, 1e-2, 0), "rollout_m0.01_after_zou_he": (trained, 1e-2, 60_000),
            "rollout_m0.001": (trained, 1e-3, 0), "logged_m0.01": (nets["paper_9x20"], 1e-2, 0),
            "zou_he": (None, 0.0, 0)}, steps=n(150_000), every=max(1, n(10_000)),
            progress=_progress)
        with open(os.path.join(RESULTS, "nn_drift.json"), "w") as f:
            json.dump(_jsonable(res), f, indent=1)
        if which == "nn_drift":
            return
    if which in ("scaling", "all"):
        res = experiments.scaling_study(nets["paper_9x20"], steps=n(150_000), progress=_progress,
                                        mass_bound=3e-4)
        with open(os.path.join(RESULTS, "scaling_study.json"), "w") as f:
            json.dump(_jsonable(res), f, indent=1)
        print(json.dumps({"scaling_rel_err": _jsonable({re: r["rel_err"] for re, r in res.items()
                                                         if isinstance(r, dict)})}), flush=True)
    if which in ("nn", "all"):
        res = experiments.outflow_study(nets, steps=n(150_000), progress=_progress,
                                        nn_switch=n(nn_switch), mass_bound=mass_bound,
                                        seeds=study_seeds)
        res = {"mass_bound": mass_bound, **res}
        with open(os.path.join(RESULTS, f"outflow_study{_suffix(mass_bound)}.json"), "w") as f:
            json.dump(_jsonable(res), f, indent=1)
        print(json.dumps({"outflow_rel_err_mean": _jsonable({re: r["rel_err_mean"]
                                                              for re, r in res.items()
                                                              if re != "mass_bound"})}), flush=True)
    if which in ("naca", "all"):
        res = experiments.naca_study(nets, steps=n(200_000), progress=_progress,
                                     nn_switch=n(nn_switch), mass_bound=mass_bound)
        res = {"mass_bound": mass_bound, **res}
        with open(os.path.join(RESULTS, f"naca_study{_suffix(mass_bound)}.json"), "w") as f:
            json.dump(_jsonable(res), f, indent=1)
        print(json.dumps({"naca_rel_err": _jsonable({a: r["rel_err"] for a, r in res.items()
                                                      if a != "mass_bound"})}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2001)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--nx", type=int, default=4096)
    ap.add_argument("--ny", type=int, default=1024)
    ap.add_argument("--precision", default="fp32", choices=list(BYTES_PER_NODE))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-nn", action="store_true")
    ap.add_argument("--no-cbc", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the FP32-vs-FP64 precision study (C_D, C_L, St)")
    ap.add_argument("--accuracy-steps", type=int, default=300_000,
                    help="steps of the FP32-vs-FP64 runs (the statistics window, the last "
                         "40 %%, must cover saturated shedding)")
    ap.add_argument("--launch", default="auto", choices=["auto", "triples", "pairs", "single"],
                    help="kernel schedule of the timed lattice (lbm_params.launch)")
    ap.add_argument("--no-big", action="store_true",
                    help="skip the 16384x4096 lattice (4.8 GB working set)")
    ap.add_argument("--big-steps", type=int, default=402)
    ap.add_argument("--no-cpu-all-cores", action="store_true")
    ap.add_argument("--study", choices=["train", "nn", "naca", "vortex", "cbc_train",
                                        "cbc_train_mach", "nn_train", "nn_drift", "scaling",
                                        "all"],
                    default=None,
                    help="also run the truncated-domain outflow study (training data, "
                         "training, neural vs Zou-He outflow) and/or the NACA0012 study; "
                         "results go to results/<study>.json")
    ap.add_argument("--study-scale", type=float, default=1.0,
                    help="fraction of the study step counts (for quick checks)")
    ap.add_argument("--study-seeds", default="2",
                    help="seeds of the initial noise for the truncated-domain study (comma-separated)")
    ap.add_argument("--nn-mass-bound", type=float, default=1e-2,
                    help="fallback density bound of the neural outflow in the studies")
    ap.add_argument("--nn-switch", type=int, default=0,
                    help="steps of Zou & He before the neural outflow is switched on (studies)")
    ap.add_argument("--no-cbc-train", action="store_true",
                    help="skip timing the closed-loop trainer of the CBC tuning network")
    ap.add_argument("--no-3d", action="store_true", help="skip the D3Q19 step")
    ap.add_argument("--no-batch", action="store_true", help="skip the training-data batch")
    ap.add_argument("--calibration-copy", action="store_true")
    ap.add_argument("--write-traffic", nargs=4, metavar="CSV")
    args = ap.parse_args()
    if args.calibration_copy:
        return calibration_copy()
    if args.write_traffic:
        return write_traffic(args.nx, args.ny, *args.write_traffic,
                             command_note=os.environ.get("TRAFFIC_NOTE", ""))
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the lattice would shard in x-slabs with a per-step halo exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_05293_amd import lbm
    nx, ny = args.nx, args.ny
    mask, tau = c2_case(nx, ny)
    kw = dict(precision=args.precision, collision="mrt", lateral="walls", u_in=0.05,
              noise_amp=1e-4, seed=2, s_e=1.0, s_eps=1.0, s_q=1.0)
    lat = lbm.Lattice(mask, tau, launch=args.launch, **kw)
    ms = time_steps(lat, args.steps, args.warmup, torch)
    out = lat.forces()
    assert out.nonfinite == 0
    nodes = nx * ny
    mlups = nodes / (ms * 1e-3) / 1e6
    # steps per launch of the Zou & He lattice: three by default at FP32 and
    # FP16 (lbm_params.launch), two at FP64 or with --launch pairs
    spl = {"single": 1, "pairs": 2}.get(args.launch, 2 if args.precision == "fp64" else 3)
    counted = args.precision == "fp32" and spl == STEPS_PER_LAUNCH
    roofline = step_roofline(nodes, ms, spl, args.precision,
                             stored_traffic(nx, ny) if counted else None)

    nn = None
    if not args.no_nn:
        lat.set_outflow_nn(random_mlp(), mass_bound=1e-2)
        ms_nn = time_steps(lat, args.steps, args.warmup, torch)
        out_nn = lat.forces()
        del lat
        single = lbm.Lattice(mask, tau, launch="single", **kw)
        ms_single = time_steps(single, args.steps, args.warmup, torch)
        del single
        two = lbm.Lattice(mask, tau, launch="pairs", **kw)
        ms_two = time_steps(two, args.steps, args.warmup, torch)
        del two
        nn = {"mlups": nodes / (ms_nn * 1e-3) / 1e6, "ms_per_step": ms_nn,
              "ratio_to_zouhe": ms / ms_nn, "ratio_to_zouhe_pairs": ms_two / ms_nn,
              "ratio_to_zouhe_single": ms_single / ms_nn,
              "zouhe_pairs_mlups": nodes / (ms_two * 1e-3) / 1e6,
              "zouhe_single_mlups": nodes / (ms_single * 1e-3) / 1e6,
              "weights": "random-init 27-64-64-3", "fallback_nodes": int(out_nn.n_fallback),
              "note": "ratio_to_zouhe: against the Zou & He lattice on the timed schedule "
                      "(three steps per launch for both); ratio_to_zouhe_pairs: against Zou & "
                      "He at two steps per launch; ratio_to_zouhe_single: one launch per step"}
    else:
        del lat
    cbc = None
    if not args.no_cbc:
        # the characteristic outflow takes periodic laterals: the same lattice
        # with periodic laterals, Zou & He then characteristic outlet
        cs = 3 ** -0.5
        kwp = dict(kw, lateral="periodic")
        lat = lbm.Lattice(mask, tau, launch=args.launch, **kwp)
        ms_zh = time_steps(lat, args.steps, args.warmup, torch)
        lat.set_outflow_cbc(sigma=0.25, kappa2=0.05 / cs, mach=0.05 / cs)
        ms_cbc = time_steps(lat, args.steps, args.warmup, torch)
        assert lat.forces().nonfinite == 0
        del lat
        two = lbm.Lattice(mask, tau, launch="pairs", **kwp)
        ms_zh2 = time_steps(two, args.steps, args.warmup, torch)
        del two
        cbc = {"mlups": nodes / (ms_cbc * 1e-3) / 1e6, "ms_per_step": ms_cbc,
               "ratio_to_zouhe": ms_zh / ms_cbc, "ratio_to_zouhe_pairs": ms_zh2 / ms_cbc,
               "zouhe_mlups": nodes / (ms_zh * 1e-3) / 1e6,
               "zouhe_pairs_mlups": nodes / (ms_zh2 * 1e-3) / 1e6,
               "setting": "same lattice with periodic laterals; characteristic outflow, "
                          "sigma 0.25, kappa_2 = Ma; ratio_to_zouhe against Zou & He on the "
                          "timed schedule (three steps per launch for both), "
                          "ratio_to_zouhe_pairs against Zou & He at two steps per launch"}
    big = None
    if not args.no_big:
        bx, by = 16384, 4096
        bmask, btau = c2_case(bx, by)
        lat = lbm.Lattice(bmask, btau, launch=args.launch, **kw)
        ms_big = time_steps(lat, args.big_steps, 20, torch)
        assert lat.forces().nonfinite == 0
        del lat
        torch.cuda.empty_cache()
        big = {"workload": f"same physics at {bx}x{by} (D = {80 * bx // 4096}), "
                           f"{BYTES_PER_NODE[args.precision] * bx * by / 1e9:.1f} GB per step of "
                           "population traffic, far above the 256 MB cache",
               "mlups": bx * by / (ms_big * 1e-3) / 1e6, "ms_per_step": ms_big,
               "steps": args.big_steps,
               "roofline": step_roofline(bx * by, ms_big, spl, args.precision,
                                         stored_traffic(bx, by) if counted else None)}
    torch.cuda.synchronize()
    cbc_training = None if args.no_cbc_train else time_cbc_training(torch)
    d3q19 = None if args.no_3d else time_d3q19(torch)
    batch = None if args.no_batch else time_batch(torch)

    accuracy = None
    if not args.no_accuracy:
        from paper_2506_05293_amd import experiments
        acc = experiments.precision_study(args.accuracy_steps, nx, ny)
        keys = ("cd_mean", "cl_rms", "st", "mlups", "cl_rms_halves")
        h = acc["fp64"]["cl_rms_halves"]
        accuracy = {"workload": f"same lattice, {args.accuracy_steps} steps, FP32 offsets vs FP64, "
                                "statistics over the last 40 %",
                    "fp32": {k: acc["fp32"].get(k) for k in keys},
                    "fp64": {k: acc["fp64"].get(k) for k in keys},
                    "rel_err": acc["rel_err"],
                    "gates": {"cd_mean": 5e-3, "cl_rms": 5e-3, "st": 1e-2},
                    "pass": all(acc["rel_err"][k] <= g for k, g in
                                (("cd_mean", 5e-3), ("cl_rms", 5e-3), ("st", 1e-2))),
                    # saturated shedding: the rms of C_L - mean agrees between
                    # the two halves of the window
                    "cl_rms_half_change": abs(h[1] - h[0]) / h[1]}
    if args.study:
        run_studies(args.study, args.study_scale, args.nn_switch, args.nn_mass_bound,
                    tuple(int(v) for v in args.study_seeds.split(",")))

    line = {
        "metric": "MLUPS + %HBM peak; C_D/C_L/St error, NN vs Zou-He outflow at same MLUPS",
        "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16-storage/f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"D2Q9 MRT channel {nx}x{ny}, cylinder D={80 * nx // 4096} at x=10D, "
                               f"{args.precision} offset storage, Zou-He inlet/outlet, walls, Re=200",
                   "nx": nx, "ny": ny, "precision": args.precision, "collision": "mrt"},
        "roofline": roofline,
        "c2_big": big,
        "nn_outflow": nn,
        "cbc_outflow": cbc,
        "cbc_training": cbc_training,
        "d3q19": d3q19,
        "batch": batch,
        "accuracy": accuracy,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(
            nx, ny, all_cores=not args.no_cpu_all_cores),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
