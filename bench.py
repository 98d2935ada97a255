"""Throughput of the fused D2Q9 step on one MI355X.

Workload (default): the 4096 x 1024 channel with a cylinder of D = 80 at
x = 10 D, MRT collision, populations stored as FP32 offsets f - w, Zou & He
velocity inlet and pressure outlet, bounce-back walls, Re = 200, seeded
velocity noise 1e-4.  One step = one pass of the whole hot path: pull
streaming with half-way bounce-back, inlet and outlet columns, collision,
momentum-exchange force and mass reduction.  The same lattice is then timed
with the neural outflow active (MLP 27-64-64-3 fused into the step).

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_NODE = {"fp64": 144, "fp32": 72, "fp16": 36}   # 9 loads + 9 stores
HBM_PEAK_GBS = 8000.0


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


def cpu_baseline(nx, ny, seconds=15.0):
    """The FP64 oracle (single thread) on the same lattice for as many whole
    steps as fit in ~`seconds` (at least one)."""
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
        dt = time.perf_counter() - t0
    return {"value": nx * ny * n / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{n} steps of the same {nx}x{ny} MRT lattice, FP64 NumPy, 1 thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--nx", type=int, default=4096)
    ap.add_argument("--ny", type=int, default=1024)
    ap.add_argument("--precision", default="fp32", choices=list(BYTES_PER_NODE))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-nn", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the lattice would shard in x-slabs with a per-step halo exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_05293_amd import lbm
    nx, ny = args.nx, args.ny
    mask, tau = c2_case(nx, ny)
    lat = lbm.Lattice(mask, tau, precision=args.precision, collision="mrt", lateral="walls",
                      u_in=0.05, noise_amp=1e-4, seed=2)
    ms = time_steps(lat, args.steps, args.warmup, torch)
    out = lat.forces()
    assert out.nonfinite == 0
    nodes = nx * ny
    mlups = nodes / (ms * 1e-3) / 1e6
    bpn = BYTES_PER_NODE[args.precision]
    gbs = bpn * nodes / (ms * 1e-3) / 1e9

    nn = None
    if not args.no_nn:
        lat.set_outflow_nn(random_mlp(), mass_bound=1e-2)
        ms_nn = time_steps(lat, args.steps, args.warmup, torch)
        out_nn = lat.forces()
        nn = {"mlups": nodes / (ms_nn * 1e-3) / 1e6, "ms_per_step": ms_nn,
              "ratio_to_zouhe": ms / ms_nn, "weights": "random-init 27-64-64-3",
              "fallback_nodes": int(out_nn.n_fallback)}
    del lat
    torch.cuda.synchronize()

    line = {
        "metric": "MLUPS + %HBM peak; C_D/C_L/St error, NN vs Zou-He outflow at same MLUPS",
        "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16-storage/f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"D2Q9 MRT channel {nx}x{ny}, cylinder D={80 * nx // 4096} at x=10D, "
                               f"{args.precision} offset storage, Zou-He inlet/outlet, walls, Re=200",
                   "nx": nx, "ny": ny, "precision": args.precision, "collision": "mrt"},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_node": bpn, "kernel": "k_step (fused pull stream-collide)"},
        "hbm_fraction": gbs / HBM_PEAK_GBS,
        "nn_outflow": nn,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(nx, ny),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
