#!/usr/bin/env python3
"""Throughput of the fused D3Q27 cascaded-LBM step on one MI355X.

Workload (the roofline and precision case): Kolmogorov-forced flow on a 512^3
periodic lattice, F_x = 1e-5 sin(2 pi 4 y / 512) as a per-node FP32 field,
nu = 0.005, seeded U(-1e-3, 1e-3) velocity perturbation, populations stored as
FP32 deviations f - w with FP32 arithmetic.  A "step" is one time step of the
whole lattice (pairs of steps run as one launch of the fused two-step
collide-and-stream kernel); the metric is MLUPS (million lattice-node updates
per second) and the fraction of the HBM roofline.  Inputs are resident in HBM
before the timed region.

Also reported from the same run (each timed with HIP events, trimmed mean of
9 repetitions as in the paper's Table I protocol): the single-step kernel and
dense planes on the same lattice; FP64, FP16 and BF16 storage; the MRT of
Appendix B and the D3Q19 scheme of Appendix A; the lid-driven cavity 256^3;
Table I's shear-wave workload (cascaded against SRT, also from HIP graph
replays); the 128^3 Taylor-Green case; the porous duct 640x320x320; the
adjoint step and the end-to-end gradient on its 256x128x128 crop and on the
64^3 channel; the velocity error of every storage type against FP64 after
500 steps; and the FP64 CPU oracle on bounded samples.

Prints one JSON line on stdout; progress goes to stderr.
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD datasheet
PMC_SINGLE = os.path.join(ROOT, "profiles", "pmc_k_step_f32_kolmogorov512.json")
PMC_FUSED = os.path.join(ROOT, "profiles", "pmc_k_step2_f32_kolmogorov512.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1801_04586_amd", "csrc", f) for f in ("node.hpp", "kernels.hpp")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def bytes_per_node(storage: str, field: bool, solid: bool, q: int = 27) -> int:
    size = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[storage]
    b = 2 * q * size
    if field:
        b += 3 * (8 if storage == "f64" else 4)
    if solid:
        b += 1
    return b


def pmc_traffic(path: str, size: int, fused: bool):
    """HBM bytes per launch from a committed counter summary, if it was taken on
    the current kernel source, lattice size and launch kind; else None."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        pmc = json.load(fh)
    if pmc.get("kernel_src_sha") == kernel_sha() and pmc.get("size") == size and pmc.get("fused") == fused:
        return pmc.get("hbm_bytes_per_launch")
    return None


def trimmed_mean(xs):
    xs = sorted(xs)
    if len(xs) > 2:
        xs = xs[1:-1]
    return sum(xs) / len(xs)


def time_steps(torch, lat, steps, reps=9):
    """Trimmed-mean ms per step over `reps` repetitions of `steps` steps (HIP events)."""
    out = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        lat.step(steps)
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b) / steps)
    return trimmed_mean(out)


def graph_of_steps(torch, lat, steps):
    """A HIP graph (torch.cuda.CUDAGraph) of lat.step(steps), captured on a side stream.  With an even
    number of launches the state ends in the buffer it started in, so every replay advances it."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            lat.step(steps)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    return graph


def kolmogorov_inputs(dims):
    import workloads

    u0 = workloads.uniform_random_velocity(dims, 1e-3, workloads.SEED)
    F = workloads.kolmogorov_force(dims, 1e-5, 4)
    return u0, F


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--size", type=int, default=512, help="edge of the cubic Kolmogorov lattice")
    ap.add_argument("--primary-only", action="store_true", help="time only the FP32 step (for profilers)")
    ap.add_argument("--copy-calibration", action="store_true", help="also run the plain copy kernel (PMC scale)")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_1801_04586_amd import Lattice

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L = args.size
    dims = (L, L, L)
    nodes = L ** 3
    nu = 0.005
    rates = workloads.rates(nu)
    log(f"[bench] Kolmogorov {dims}, nu={nu}, s2={rates[2]:.6f}; generating inputs")
    u0, F = kolmogorov_inputs(dims)
    u0_dev = torch.from_numpy(u0).to(dev)
    F32_dev = torch.from_numpy(F).to(dev, torch.float32)
    F64_dev = None

    # ------------------------------------------------------------------ primary: FP32 storage
    lat = Lattice(dims, (0, 0, 0), "f32", rates, force_field=F32_dev, device=dev)
    lat.init(None, u0_dev)
    lat.step(args.warmup)
    torch.cuda.synchronize()
    fused = lat.uses_fused_pairs
    launches = (args.steps // 2 + args.steps % 2) if fused else args.steps
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    lat.step(args.steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    event_ms = ev0.elapsed_time(ev1)
    kernel_ms = event_ms / launches
    ms_per_step = wall * 1e3 / args.steps
    mlups = nodes * args.steps / wall / 1e6
    bpn = bytes_per_node("f32", True, False)
    # algorithmic bytes of the node updates done in the timed region, per unit of kernel time
    achieved = bpn * nodes * args.steps / (event_ms * 1e-3) / 1e9
    log(f"[bench] f32 ({'two fused steps per launch' if fused else 'one step per launch'}): {ms_per_step:.3f} "
        f"ms/step wall, {kernel_ms:.3f} ms/launch, {mlups:.0f} MLUPS, {achieved:.0f} GB/s algorithmic")
    _, _, tot, nbad = lat.moments(fields=False)
    if nbad:
        log(f"[bench] WARNING: {nbad} non-finite nodes")

    if args.copy_calibration:
        tmp = torch.empty_like(lat.state)
        for _ in range(5):
            lat.ctx.copy(lat.state, tmp)
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(5):
            lat.ctx.copy(lat.state, tmp)
        c1.record()
        torch.cuda.synchronize()
        cms = c0.elapsed_time(c1) / 5
        log(f"[bench] copy {lat.state.numel() * 4 / 1e9:.2f} GB: {cms:.3f} ms = "
            f"{2 * lat.state.numel() * 4 / (cms * 1e-3) / 1e9:.0f} GB/s read+write")
        del tmp

    traffic = pmc_traffic(PMC_FUSED if fused else PMC_SINGLE, L, fused)
    kname = "k_step2<float, force field> (two fused steps)" if fused else "k_step<float, periodic, force field>"

    result = {
        # the headline metric; value = FP32-storage MLUPS of the fused D3Q27 cascaded step, roofline.frac its
        # HBM fraction; FP64/FP16/BF16 storage, the adjoint and the errors against FP64 are under variants
        # and accuracy_vs_f64
        "metric": "MLUPS & % HBM roofline: FP64 vs FP32/FP16-storage fwd, adjoint MLUPS, at stated err",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"kolmogorov_{L}^3",
            "nodes": nodes,
            "storage": "f32 deviations f - w",
            "force": "per-node FP32 field, F0 = 1e-5, k = 4",
            "nu": nu,
            "boundaries": "periodic",
            "bytes_per_node": bpn,
            "plane_stride": lat.P,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": kname,
            "kernel_ms": round(kernel_ms, 4),
            "node_updates_per_launch": nodes * (2 if fused else 1),
            "algorithmic_bytes_per_launch": bpn * nodes * (2 if fused else 1),
            # HBM bytes the kernel actually moves (counter summary) per unit of kernel time; with two
            # fused steps per launch this is below the algorithmic rate, which counts every update
            "traffic_gbs": None if traffic is None else round(traffic / (kernel_ms * 1e-3) / 1e9, 1),
            "traffic_frac": None if traffic is None else round(traffic / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        },
    }
    if fused:
        # the same lattice with one step per launch, for comparison
        lat.set_fused_steps(False)
        ms1 = time_steps(torch, lat, 10)
        lat.set_fused_steps(None)
        result["single_step_kernel"] = {
            "mlups": round(nodes / (ms1 * 1e-3) / 1e6, 1), "kernel_ms": round(ms1, 4),
            "frac": round(bpn * nodes / (ms1 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": pmc_traffic(PMC_SINGLE, L, False)}
        log(f"[bench] f32 single steps: {result['single_step_kernel']}")
    if args.primary_only:
        print(json.dumps(result), flush=True)
        return

    # the same workload with dense planes (plane stride = N, a power of two here)
    ld = Lattice(dims, (0, 0, 0), "f32", rates, force_field=F32_dev, device=dev, plane_stride=0)
    ld.init(None, u0_dev)
    ld.step(4)
    msd = time_steps(torch, ld, 10)
    ld.set_fused_steps(False)
    msd1 = time_steps(torch, ld, 10)
    result["dense_planes"] = {"plane_stride": ld.P, "fused_mlups": round(nodes / (msd * 1e-3) / 1e6, 1),
                              "single_step_mlups": round(nodes / (msd1 * 1e-3) / 1e6, 1)}
    log(f"[bench] dense planes: {result['dense_planes']}")
    ld.close()
    del ld

    lat.close()
    del lat
    torch.cuda.empty_cache()

    # ------------------------------------------------------------------ other storage types, same lattice
    variants = {}
    if not args.no_variants:
        for storage in ("f64", "f16", "bf16"):
            field = F32_dev
            if storage == "f64":
                F64_dev = torch.from_numpy(F).to(dev)
                field = F64_dev
            lv = Lattice(dims, (0, 0, 0), storage, rates, force_field=field, device=dev)
            lv.init(None, u0_dev)
            lv.step(3)
            ms = time_steps(torch, lv, 10)
            b = bytes_per_node(storage, True, False)
            variants[f"kolmogorov_{L}_{storage}"] = {
                "mlups": round(nodes / (ms * 1e-3) / 1e6, 1), "kernel_ms": round(ms, 4),
                "launch": "two fused steps" if lv.uses_fused_pairs else "one step",
                "bytes_per_node": b, "frac": round(b * nodes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            if lv.uses_fused_pairs:
                lv.set_fused_steps(False)
                ms1 = time_steps(torch, lv, 10)
                lv.set_fused_steps(None)
                variants[f"kolmogorov_{L}_{storage}"]["single_step_mlups"] = round(nodes / (ms1 * 1e-3) / 1e6, 1)
            log(f"[bench] {storage}: {ms:.3f} ms/step, {variants[f'kolmogorov_{L}_{storage}']}")
            lv.close()
            del lv
            torch.cuda.empty_cache()
        # the raw-moment MRT of Appendix B (Guo forcing) on the same lattice and force field, FP32
        lv = Lattice(dims, (0, 0, 0), "f32", rates, force_field=F32_dev, device=dev, collision="mrt")
        lv.init(None, u0_dev)
        lv.step(4)
        ms = time_steps(torch, lv, 10)
        b = bytes_per_node("f32", True, False)
        variants[f"kolmogorov_{L}_mrt_f32"] = {
            "mlups": round(nodes / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
            "launch": "two fused steps" if lv.uses_fused_pairs else "one step", "bytes_per_node": b,
            "frac": round(b * nodes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"[bench] MRT f32: {variants[f'kolmogorov_{L}_mrt_f32']}")
        lv.close()
        del lv
        torch.cuda.empty_cache()

        # the D3Q19 scheme of Appendix A on the same lattice and force field
        for storage in ("f32", "f64", "f16"):
            field = F32_dev if storage != "f64" else F64_dev
            lv = Lattice(dims, (0, 0, 0), storage, rates, force_field=field, device=dev, lattice="d3q19")
            lv.init(None, u0_dev)
            lv.step(3)
            ms = time_steps(torch, lv, 10)
            b = bytes_per_node(storage, True, False, q=19)
            key = f"kolmogorov_{L}_d3q19_{storage}"
            variants[key] = {"mlups": round(nodes / (ms * 1e-3) / 1e6, 1), "kernel_ms": round(ms, 4),
                             "bytes_per_node": b, "frac": round(b * nodes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            log(f"[bench] D3Q19 {storage}: {variants[key]}")
            lv.close()
            del lv
            torch.cuda.empty_cache()
        step_ms = event_ms / args.steps
        variants[f"kolmogorov_{L}_f32"] = {"mlups": round(nodes / (step_ms * 1e-3) / 1e6, 1),
                                           "ms_per_step": round(step_ms, 4), "bytes_per_node": bpn,
                                           "frac": round(achieved / HBM_PEAK_GBS, 4)}
        f64k = variants[f"kolmogorov_{L}_f64"]["kernel_ms"]
        result["speedup_f32_over_f64"] = round(f64k / step_ms, 3)

        # lid-driven cavity 256^3 (all walls, lid moving with U = 0.1), cascaded and MRT, FP32: the walled path
        cdims = (256, 256, 256)
        for coll in ("cascaded", "mrt"):
            lv = Lattice(cdims, (1, 1, 1), "f32", workloads.rates(0.1 * 256 / 400.0), device=dev, collision=coll,
                         wall_velocity={(1, 1): (0.1, 0.0, 0.0)})
            lv.init()
            lv.step(3)
            ms = time_steps(torch, lv, 10)
            b = bytes_per_node("f32", False, False)
            variants[f"cavity_256_{coll}_f32"] = {
                "mlups": round(256 ** 3 / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
                "launch": "two fused steps" if lv.uses_fused_pairs else "one step", "bytes_per_node": b,
                "frac": round(b * 256 ** 3 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            if lv.uses_fused_pairs:
                lv.set_fused_steps(False)
                ms1 = time_steps(torch, lv, 10)
                variants[f"cavity_256_{coll}_f32"]["single_step_mlups"] = round(256 ** 3 / (ms1 * 1e-3) / 1e6, 1)
            log(f"[bench] cavity {coll}: {variants[f'cavity_256_{coll}_f32']}")
            lv.close()
            del lv
        torch.cuda.empty_cache()

        # Table I's workload: 10 000 steps of the shear wave on 5 x ny x 5, the cascaded scheme against
        # the SRT (BGK) LBM with the discrete equilibrium -- the MRT with every rate equal -- in FP64
        table1 = {}
        for ny in (101, 201, 401):
            sdims = (5, ny, 5)
            phi = 2 * np.pi / ny
            us = np.zeros((3, 5, ny, 5))
            us[0] = (1e-3 * np.sin(phi * np.arange(ny)))[None, :, None]
            us[1] = 0.3 / np.sqrt(3.0)
            row = {}
            for name, coll, r in (("t_C", "cascaded", workloads.rates(0.05)),
                                  ("t_S", "mrt", np.full(10, workloads.s2_from_nu(0.05)))):
                lv = Lattice(sdims, (0, 0, 0), "f64", r, device=dev, collision=coll)
                lv.init(None, us)
                lv.step(100)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lv.step(10000)
                torch.cuda.synchronize()
                row[name] = round(time.perf_counter() - t0, 5)
                # the same 10 000 steps as 100 replays of a HIP graph of 100 launches (launch-bound lattices)
                graph = graph_of_steps(torch, lv, 100)
                graph.replay()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(100):
                    graph.replay()
                torch.cuda.synchronize()
                row[name + "_graph"] = round(time.perf_counter() - t0, 5)
                del graph
                lv.close()
            row["t_C/t_S"] = round(row["t_C"] / row["t_S"], 3)
            row["t_C/t_S_graph"] = round(row["t_C_graph"] / row["t_S_graph"], 3)
            table1[f"5x{ny}x5"] = row
        variants["table_I_shear_wave_10000_steps_f64"] = table1
        log(f"[bench] Table I workload: {table1}")

        # plain kernel on the 128^3 Taylor-Green case
        tdims = (128, 128, 128)
        rho_t, u_t = workloads.taylor_green_3d(tdims, 0.04)
        for storage in ("f64", "f32"):
            lt = Lattice(tdims, (0, 0, 0), storage, workloads.rates(0.01), device=dev)
            lt.init(rho_t, u_t)
            lt.step(3)
            ms = time_steps(torch, lt, 50)
            b = bytes_per_node(storage, False, False)
            variants[f"taylor_green_128_{storage}"] = {
                "mlups": round(128 ** 3 / (ms * 1e-3) / 1e6, 1), "kernel_ms": round(ms, 4), "bytes_per_node": b,
                "frac": round(b * 128 ** 3 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "note": "2 x 226-453 MB working set: partly served by the 256 MB last-level cache"}
            lt.close()

        # porous duct 640x320x320, FP32, walls in y and z, spheres (solid fraction 0.2)
        pdims = (640, 320, 320)
        pmask, _, _ = workloads.porous_spheres(pdims, (0, 1, 1), 6.0, 12.0, 0.2, workloads.SEED)
        lp = Lattice(pdims, (0, 1, 1), "f32", workloads.rates(0.02), force=(2e-6, 0, 0), solid=pmask, device=dev)
        lp.init()
        lp.step(3)
        ms = time_steps(torch, lp, 10)
        pn = int(np.prod(pdims))
        fluid = int((pmask == 0).sum())
        pb = 2 * 27 * 4 * fluid + pn  # populations of fluid nodes + the solid mask
        variants["porous_640x320x320_f32"] = {
            "mlups": round(pn / (ms * 1e-3) / 1e6, 1), "mflups_fluid": round(fluid / (ms * 1e-3) / 1e6, 1),
            "ms_per_step": round(ms, 4), "launch": "two fused steps" if lp.uses_fused_pairs else "one step",
            "bytes_per_node": round(pb / pn, 2),
            "frac": round(pb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "solid_fraction": round(1 - fluid / pn, 4)}
        if lp.uses_fused_pairs:
            lp.set_fused_steps(False)
            ms1 = time_steps(torch, lp, 10)
            variants["porous_640x320x320_f32"]["single_step_mlups"] = round(pn / (ms1 * 1e-3) / 1e6, 1)
        log(f"[bench] porous: {variants['porous_640x320x320_f32']}")
        lp.close()
        del lp
        torch.cuda.empty_cache()

        # end-to-end gradient on the adjoint channel case: 64^3, T = 200, checkpoint every 20, FP32
        from paper_1801_04586_amd.adjoint import flow_loss

        cdims, T, K = (64, 64, 64), 200, 20
        Fc = workloads.gaussian_force(cdims, 1e-6, workloads.SEED)
        lc = Lattice(cdims, (0, 1, 0), "f32", workloads.rates(0.05), force_field=Fc, device=dev)
        lc.init()
        s0 = lc.state.clone()
        utc = torch.from_numpy(workloads.channel_target(cdims, (0, 1, 0), 1e-4)).to(dev, torch.float32)
        Ft = torch.from_numpy(Fc).to(dev, torch.float32)
        st = torch.from_numpy(workloads.rates(0.05))
        times = []
        for _ in range(3):
            Fr, sr = Ft.clone().requires_grad_(True), st.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            flow_loss(Fr, sr, lc, s0, utc, T, K).backward()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        cn = int(np.prod(cdims))
        tbest = min(times)
        variants["adjoint_channel_64_f32_T200_K20"] = {
            "gradient_seconds": round(tbest, 4),
            "node_updates_per_s_M": round(cn * T * 3 / tbest / 1e6, 1),
            "note": "forward T steps + recompute T steps + T adjoint steps, 64^3 (cache-resident, launch-bound)"}
        log(f"[bench] adjoint channel: {variants['adjoint_channel_64_f32_T200_K20']}")
        lc.close()

        # adjoint step on a porous crop (FP32, walls y/z, spheres, per-node force field)
        adims = (256, 128, 128)
        mask, _, _ = workloads.porous_spheres(adims, (0, 1, 1), 6.0, 12.0, 0.2, workloads.SEED)
        Fa = workloads.gaussian_force(adims, 1e-6, workloads.SEED)
        la = Lattice(adims, (0, 1, 1), "f32", workloads.rates(0.02), force=(2e-6, 0, 0), force_field=Fa, solid=mask,
                     device=dev)
        la.init()
        la.step(5)
        ut = torch.zeros((3,) + la.shape, dtype=torch.float32, device=dev)
        lam = torch.empty((27,) + la.shape, dtype=torch.float32, device=dev)
        lam2 = torch.empty_like(lam)
        gF = torch.zeros((3,) + la.shape, dtype=torch.float32, device=dev)
        gs = torch.zeros(10, dtype=torch.float64, device=dev)
        la.ctx.loss_seed(la.state, ut, lam, gF, None)
        an = int(np.prod(adims))
        reps = []
        for _ in range(9):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(10):
                la.ctx.adjoint_step(la.state, lam, lam2, gF, gs)
                lam, lam2 = lam2, lam
            b.record()
            b.synchronize()
            reps.append(a.elapsed_time(b) / 10)
        ams = trimmed_mean(reps)
        fwd = time_steps(torch, la, 10)
        # adjoint bytes per fluid node: state 27x4 + lambda in/out 2x27x4 + dJ/dF rmw 2x3x4 + force 3x4 + mask
        ab = 27 * 4 * 3 + 24 + 12 + 1
        variants["adjoint_porous_256x128x128_f32"] = {
            "adjoint_mlups": round(an / (ams * 1e-3) / 1e6, 1), "adjoint_kernel_ms": round(ams, 4),
            "with_recompute_mlups": round(an / ((ams + fwd) * 1e-3) / 1e6, 1),
            "bytes_per_node": ab, "frac": round(ab * an / (ams * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "solid_fraction": round(float(mask.mean()), 4)}
        log(f"[bench] adjoint: {variants['adjoint_porous_256x128x128_f32']}")
        # end to end: gradient of the flow loss on the crop, T = 40 steps, checkpoint every K = 20
        from paper_1801_04586_amd.adjoint import flow_loss

        Ta, Ka = 40, 20
        s0a = la.state.clone()
        Fta = torch.from_numpy(Fa).to(dev, torch.float32)
        sta = torch.from_numpy(workloads.rates(0.02))
        times = []
        for _ in range(3):
            Fr, sr = Fta.clone().requires_grad_(True), sta.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            flow_loss(Fr, sr, la, s0a, ut, Ta, Ka).backward()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        tg = min(times)
        variants["adjoint_porous_256x128x128_f32"].update({
            "gradient_T40_K20_seconds": round(tg, 4),
            "gradient_node_updates_per_s_M": round(an * Ta * 3 / tg / 1e6, 1)})
        log(f"[bench] adjoint gradient: {variants['adjoint_porous_256x128x128_f32']}")
        la.close()
        del la, lam, lam2, gF
        torch.cuda.empty_cache()
    result["variants"] = variants

    # ------------------------------------------------------------------ accuracy of storage types vs FP64
    if not args.no_accuracy:
        steps = 500
        acc = {}
        if F64_dev is None:
            F64_dev = torch.from_numpy(F).to(dev)
        l64 = Lattice(dims, (0, 0, 0), "f64", rates, force_field=F64_dev, device=dev)
        l64.init(None, u0_dev)
        l64.step(steps)
        _, u64, _, _ = l64.moments()
        l64.close()
        del l64
        torch.cuda.empty_cache()
        nrm = torch.linalg.vector_norm(u64).item()
        umax = u64.abs().max().item()
        for storage in ("f32", "f16", "bf16"):
            ls = Lattice(dims, (0, 0, 0), storage, rates, force_field=F32_dev, device=dev)
            ls.init(None, u0_dev)
            ls.step(steps)
            _, us, _, nb = ls.moments()
            d = us - u64
            acc[storage] = {"l2_rel": float(torch.linalg.vector_norm(d).item() / nrm),
                            "max_rel": float(d.abs().max().item() / umax), "nonfinite": int(nb)}
            log(f"[bench] accuracy {storage} after {steps} steps: {acc[storage]}")
            ls.close()
            del ls, us, d
            torch.cuda.empty_cache()
        acc["reference"] = f"FP64 storage, same inputs, {steps} steps; u_max = {umax:.4e}"
        result["accuracy_vs_f64"] = acc
        del u64

    # ------------------------------------------------------------------ CPU oracle on a bounded sample
    if not args.no_cpu:
        import oracle

        wd = (128, 128, 32)
        g = oracle.Geometry(dims, (0, 0, 0), (0, 0, 0), wd)
        sl = (slice(0, wd[2]), slice(0, wd[1]), slice(0, wd[0]))
        f0 = oracle.init(g, None, np.ascontiguousarray(u0[(slice(None),) + sl]))
        Fw = np.ascontiguousarray(F[(slice(None),) + sl])
        t0 = time.perf_counter()
        f = oracle.step(g, f0, rates, force_field=Fw)
        t1 = time.perf_counter() - t0
        nsteps = max(1, min(50, int(args.cpu_seconds / max(t1, 1e-3))))
        t0 = time.perf_counter()
        for _ in range(nsteps):
            f = oracle.step(g, f, rates, force_field=Fw)
        tc = time.perf_counter() - t0
        wn = int(np.prod(wd))
        result["cpu_baseline"] = {
            "value": round(wn * nsteps / tc / 1e6, 4), "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{wd[0]}x{wd[1]}x{wd[2]} window of the {L}^3 Kolmogorov lattice, {nsteps} steps, FP64 dense "
                      f"27x27 oracle, {tc:.1f} s"}
        budget = args.cpu_seconds / 2

        def timed_run(geom, f, rates_, max_steps, **kw):
            # one step to size the run, then as many as fit the budget (at most max_steps)
            t0 = time.perf_counter()
            f = oracle.step(geom, f, rates_, **kw)
            t1 = time.perf_counter() - t0
            n = max(1, min(max_steps, int(budget / max(t1, 1e-4))))
            t0 = time.perf_counter()
            for _ in range(n):
                f = oracle.step(geom, f, rates_, **kw)
            dt = time.perf_counter() - t0
            return geom.n * n / dt / 1e6, n, dt

        # one core, a smaller window of the same workload
        nthreads = oracle.num_threads()
        oracle.set_num_threads(1)
        w1 = (64, 64, 16)
        g1 = oracle.Geometry(dims, (0, 0, 0), (0, 0, 0), w1)
        s1 = (slice(0, w1[2]), slice(0, w1[1]), slice(0, w1[0]))
        f1 = oracle.init(g1, None, np.ascontiguousarray(u0[(slice(None),) + s1]))
        m1, n1, d1 = timed_run(g1, f1, rates, 50, force_field=np.ascontiguousarray(F[(slice(None),) + s1]))
        oracle.set_num_threads(nthreads)
        result["cpu_baseline"]["single_core"] = {
            "value": round(m1, 4), "cores": 1,
            "sample": f"{w1[0]}x{w1[1]}x{w1[2]} window of the same lattice, {n1} steps, {d1:.1f} s"}
        # the force-driven channel (16x32x16, FP64, 3000 steps) and the 128^3 Taylor-Green vortex, all cores
        pc = workloads.POISEUILLE
        gp = oracle.Geometry(pc.dims, pc.walls)
        mp, npo, dp_ = timed_run(gp, oracle.init(gp), pc.rates(), pc.steps, force=pc.force_uniform)
        tc2 = workloads.TGV128
        gt = oracle.Geometry(tc2.dims, tc2.walls)
        rt0, ut0 = workloads.taylor_green_3d(tc2.dims, 0.04)
        mt, ntg, dtg = timed_run(gt, oracle.init(gt, rt0, ut0), tc2.rates(), tc2.steps)
        result["cpu_baseline"]["other_workloads"] = {
            pc.name: {"value": round(mp, 4), "steps": npo, "seconds": round(dp_, 2)},
            tc2.name: {"value": round(mt, 4), "steps": ntg, "seconds": round(dtg, 2)}}
        log(f"[bench] cpu baseline: {result['cpu_baseline']}")

    result["context"] = {
        "paper_cpu": "0.45 MLUPS: C++ CLBM, i7-6500U laptop, 5x101x5 shear wave (Table I), context only",
        "paper_table_I_seconds": {"5x101x5": [56.028, 26.042, 2.151], "5x201x5": [111.838, 51.728, 2.162],
                                  "5x401x5": [217.027, 101.179, 2.145], "columns": "t_C, t_S, t_C/t_S (CPU)"},
        "hbm_peak_gbs": HBM_PEAK_GBS,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
