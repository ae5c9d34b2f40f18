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

Also reported from the same run (each timed with HIP events on the stream the
kernels run on, trimmed mean of 9 repetitions as in the paper's Table I
protocol) -- the variants below, by name; `--only NAME[,NAME...]` runs just
those (one lattice per process, for profilers):
  kolmogorov_512_f32_single, kolmogorov_512_f32_dense   single steps; dense planes
  kolmogorov_512_{f64,f16,bf16}                          other storage types
  kolmogorov_512_general_f32                             non-slip s3 and s2b = s2 (general collision)
  kolmogorov_512_mrt_f32, kolmogorov_512_d3q19_{f32,f64,f16}   Appendix B and Appendix A
  cavity_256_{cascaded,mrt}_f32, cavity_256_cascaded_f64   lid-driven cavity, all walls
  table_I_latency, table_I_bandwidth                     Table I's cascaded/SRT cost ratio
  taylor_green_128_{f64,f32}
  porous_640x320x320_f32, porous_640x320x320_general_f32
  adjoint_channel_64_f32                                 end-to-end gradient, T = 200, K = 20
  adjoint_porous_256x128x128_f32                         adjoint step, recompute, backward, gradient
  adjoint_porous_256x128x128_f64                         adjoint step, recompute, backward (FP64 storage)
  adjoint_porous_640x320x320_f32                         adjoint step and recompute on the full duct
plus the velocity error of every storage type against FP64 after 500 steps,
and the FP64 CPU oracle on bounded samples.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD datasheet
PMC_SINGLE = os.path.join(ROOT, "profiles", "pmc_k_step_f32_kolmogorov512.json")
PMC_FUSED = os.path.join(ROOT, "profiles", "pmc_k_step2_f32_kolmogorov512.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1801_04586_amd", "csrc", f) for f in ("node.hpp", "kernels.hpp")]
HEADLINE = "kolmogorov_512_f32"
# bytes per node of one adjoint step: state 27 x 4, lambda in and out 2 x 27 x 4, dJ/dF read and written
# 2 x 3 x 4, force field 3 x 4, solid mask 1; counted over all nodes (the kernel reads and writes whole
# lines, solid nodes included), as "frac"; "frac_fluid" counts fluid nodes only
ADJ_BYTES = 27 * 4 * 3 + 24 + 12 + 1
ADJ_BYTES_F64 = 27 * 8 * 3 + 48 + 24 + 1  # FP64 storage: state, lambda in and out, dJ/dF rmw, force, mask


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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


class Bench:
    """Shared inputs and timing helpers of one bench.py process."""

    def __init__(self, args):
        import numpy as np
        import torch

        import workloads

        self.args, self.np, self.torch, self.workloads = args, np, torch, workloads
        self.dev = torch.device("cuda:0")
        torch.cuda.set_device(self.dev)
        self.L = args.size
        self.dims = (self.L,) * 3
        self.nodes = self.L ** 3
        self._kolm = None

    # ---- timing (HIP events on torch's current stream, where the library enqueues its kernels)
    def ms(self, fn, per: int, reps: int = 9) -> float:
        """Trimmed-mean milliseconds per unit over `reps` repetitions of fn(), which does `per` units."""
        torch = self.torch
        out = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            out.append(a.elapsed_time(b) / per)
        return trimmed_mean(out)

    def step_ms(self, lat, steps: int = 10, reps: int = 9) -> float:
        return self.ms(lambda: lat.step(steps), steps, reps)

    def record(self, nodes: int, ms: float, bpn: float, **extra):
        return {"mlups": round(nodes / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
                "bytes_per_node": round(bpn, 2), "frac": round(bpn * nodes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                **extra}

    # ---- inputs
    def kolmogorov(self):
        """(u0 device FP64, F device FP32, F numpy) of the 512^3 workload, generated once."""
        if self._kolm is None:
            u0 = self.workloads.uniform_random_velocity(self.dims, 1e-3, self.workloads.SEED)
            F = self.workloads.kolmogorov_force(self.dims, 1e-5, 4)
            self._kolm = (self.torch.from_numpy(u0).to(self.dev), self.torch.from_numpy(F).to(self.dev, self.torch.float32),
                          F, u0)
        return self._kolm

    def kolmogorov_lattice(self, storage="f32", rates=None, **kw):
        from paper_1801_04586_amd import Lattice

        u0d, F32, F, _ = self.kolmogorov()
        field = self.torch.from_numpy(F).to(self.dev) if storage == "f64" else F32
        r = self.workloads.rates(0.005) if rates is None else rates
        lat = Lattice(self.dims, (0, 0, 0), storage, r, force_field=field, device=self.dev, **kw)
        lat.init(None, u0d)
        return lat

    def done(self, *lats):
        for lat in lats:
            lat.close()
        self.torch.cuda.empty_cache()


def nonslip_rates(workloads, nu):
    """The walled setting of Sec. III B: non-slip s3 = (16 - 8 s2)/(8 - s2) and s2b = s2, so the general
    collision runs (rates above second order are not all 1)."""
    s2 = workloads.s2_from_nu(nu)
    return workloads.rates(nu, s2b=s2, s3=workloads.nonslip_s3(s2))


# ------------------------------------------------------------------------------------------------ variants
def v_kolmogorov_single(b: Bench):
    lat = b.kolmogorov_lattice()
    lat.set_fused_steps(False)
    lat.step(2)
    r = b.record(b.nodes, b.step_ms(lat), bytes_per_node("f32", True, False), launch="one step",
                 traffic=pmc_traffic(PMC_SINGLE, b.L, False))
    b.done(lat)
    return r


def v_kolmogorov_dense(b: Bench):
    lat = b.kolmogorov_lattice(plane_stride=0)
    lat.step(4)
    bpn = bytes_per_node("f32", True, False)
    r = b.record(b.nodes, b.step_ms(lat), bpn, launch="two fused steps", plane_stride=lat.P)
    lat.set_fused_steps(False)
    r["single_step"] = b.record(b.nodes, b.step_ms(lat), bpn)
    b.done(lat)
    return r


def v_kolmogorov_storage(storage):
    def run(b: Bench):
        lat = b.kolmogorov_lattice(storage)
        lat.step(3)
        bpn = bytes_per_node(storage, True, False)
        r = b.record(b.nodes, b.step_ms(lat), bpn, launch="two fused steps" if lat.uses_fused_pairs else "one step")
        if lat.uses_fused_pairs:
            lat.set_fused_steps(False)
            r["single_step"] = b.record(b.nodes, b.step_ms(lat), bpn)
        b.done(lat)
        return r
    return run


def v_kolmogorov_general(b: Bench):
    """The headline lattice with the general collision (non-slip s3, s2b = s2): fused pairs and single
    steps, and the ratio of its time to the rates-one path's."""
    bpn = bytes_per_node("f32", True, False)
    out = {}
    for name, rates in (("general", nonslip_rates(b.workloads, 0.005)), ("rates_one", b.workloads.rates(0.005))):
        lat = b.kolmogorov_lattice("f32", rates)
        lat.step(4)
        fused = b.step_ms(lat)
        lat.set_fused_steps(False)
        single = b.step_ms(lat)
        out[name] = (fused, single)
        b.done(lat)
    g, one = out["general"], out["rates_one"]
    r = b.record(b.nodes, g[0], bpn, launch="two fused steps", rates="s3 = (16 - 8 s2)/(8 - s2), s2b = s2")
    r["single_step"] = b.record(b.nodes, g[1], bpn)
    r["time_over_rates_one"] = {"fused": round(g[0] / one[0], 3), "single_step": round(g[1] / one[1], 3)}
    return r


def v_kolmogorov_mrt(b: Bench):
    lat = b.kolmogorov_lattice("f32", collision="mrt")
    lat.step(4)
    bpn = bytes_per_node("f32", True, False)
    r = b.record(b.nodes, b.step_ms(lat), bpn, launch="two fused steps" if lat.uses_fused_pairs else "one step")
    if lat.uses_fused_pairs:
        lat.set_fused_steps(False)
        r["single_step"] = b.record(b.nodes, b.step_ms(lat), bpn)
    b.done(lat)
    return r


def v_kolmogorov_d3q19(storage):
    def run(b: Bench):
        lat = b.kolmogorov_lattice(storage, lattice="d3q19")
        lat.step(3)
        bpn = bytes_per_node(storage, True, False, q=19)
        r = b.record(b.nodes, b.step_ms(lat), bpn, launch="two fused steps" if lat.uses_fused_pairs else "one step")
        if lat.uses_fused_pairs:
            lat.set_fused_steps(False)
            r["single_step"] = b.record(b.nodes, b.step_ms(lat), bpn)
        b.done(lat)
        return r
    return run


def v_cavity(collision, storage="f32"):
    def run(b: Bench):
        from paper_1801_04586_amd import Lattice

        cdims = (256, 256, 256)
        n = 256 ** 3
        lat = Lattice(cdims, (1, 1, 1), storage, b.workloads.rates(0.1 * 256 / 400.0), device=b.dev,
                      collision=collision, wall_velocity={(1, 1): (0.1, 0.0, 0.0)})
        lat.init()
        lat.step(3)
        bpn = bytes_per_node(storage, False, False)
        r = b.record(n, b.step_ms(lat), bpn, launch="two fused steps" if lat.uses_fused_pairs else "one step")
        if lat.uses_fused_pairs:
            lat.set_fused_steps(False)
            r["single_step"] = b.record(n, b.step_ms(lat), bpn)
        b.done(lat)
        return r
    return run


def _shear_wave(b: Bench, dims, coll, storage, rates):
    """Table I's workload: u = (A sin(2 pi y / ny), B, 0), A = 1e-3, B = 0.3 c_s, no force."""
    from paper_1801_04586_amd import Lattice

    np = b.np
    nx, ny, nz = dims
    us = np.zeros((3, nz, ny, nx))
    us[0] = (1e-3 * np.sin(2 * np.pi * np.arange(ny) / ny))[None, :, None]
    us[1] = 0.3 / np.sqrt(3.0)
    lat = Lattice(dims, (0, 0, 0), storage, rates, device=b.dev, collision=coll)
    lat.init(None, us)
    return lat


def v_table_I_latency(b: Bench):
    """Table I's lattices (5 x ny x 5, 10 000 steps, FP64): cascaded (nu = 0.05, higher rates 1) against
    the SRT-LBM with the discrete equilibrium, run as the MRT with every rate equal.  A step here is
    one kernel of about 5 us, so these ratios measure launch latency, not collision cost."""
    torch, np = b.torch, b.np
    table = {}
    for ny in (101, 201, 401):
        row = {}
        for name, coll, r in (("t_C", "cascaded", b.workloads.rates(0.05)),
                              ("t_S", "mrt", np.full(10, b.workloads.s2_from_nu(0.05)))):
            lat = _shear_wave(b, (5, ny, 5), coll, "f64", r)
            lat.step(100)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lat.step(10000)
            torch.cuda.synchronize()
            row[name] = round(time.perf_counter() - t0, 5)
            lat.close()
        row["t_C/t_S"] = round(row["t_C"] / row["t_S"], 3)
        table[f"5x{ny}x5"] = row
    return table


def v_table_I_bandwidth(b: Bench):
    """Table I's question where the GPU is full: the same shear wave and rates on a 512^3 lattice.  The
    cascaded scheme and the SRT run with the same launch structure in FP64 and in FP32 storage: single
    steps, and both with fused pairs."""
    np = b.np
    dims = (512, 512, 512)
    out = {}
    for storage in ("f64", "f32"):
        row = {}
        for name, coll, r in (("t_C", "cascaded", b.workloads.rates(0.05)),
                              ("t_S", "mrt", np.full(10, b.workloads.s2_from_nu(0.05)))):
            lat = _shear_wave(b, dims, coll, storage, r)
            lat.set_fused_steps(False)
            lat.step(2)
            row[name + "_ms_per_step"] = round(b.step_ms(lat), 4)
            lat.set_fused_steps(None)
            lat.step(2)
            if lat.uses_fused_pairs:
                row[name + "_fused_ms_per_step"] = round(b.step_ms(lat), 4)
            b.done(lat)
        row["t_C/t_S"] = round(row["t_C_ms_per_step"] / row["t_S_ms_per_step"], 3)
        if "t_C_fused_ms_per_step" in row:
            row["t_C_fused/t_S"] = round(row["t_C_fused_ms_per_step"] / row["t_S_ms_per_step"], 3)
            row["t_C_fused/t_S_fused"] = round(row["t_C_fused_ms_per_step"] / row["t_S_fused_ms_per_step"], 3)
        row["mlups_C"] = round(b.nodes / (row["t_C_ms_per_step"] * 1e-3) / 1e6, 1)
        row["mlups_S"] = round(b.nodes / (row["t_S_ms_per_step"] * 1e-3) / 1e6, 1)
        out[storage] = row
    out["workload"] = "shear wave, 512^3 periodic, nu = 0.05, Ma = 0.3, no force"
    return out


def v_taylor_green(storage):
    def run(b: Bench):
        from paper_1801_04586_amd import Lattice

        tdims = (128, 128, 128)
        rho_t, u_t = b.workloads.taylor_green_3d(tdims, 0.04)
        lat = Lattice(tdims, (0, 0, 0), storage, b.workloads.rates(0.01), device=b.dev)
        lat.init(rho_t, u_t)
        lat.step(3)
        bpn = bytes_per_node(storage, False, False)
        r = b.record(128 ** 3, b.step_ms(lat, 50), bpn, launch="two fused steps" if lat.uses_fused_pairs else "one step",
                     note="2 x 226-453 MB working set: partly served by the 256 MB last-level cache")
        if lat.uses_fused_pairs:
            lat.set_fused_steps(False)
            r["single_step"] = b.record(128 ** 3, b.step_ms(lat, 50), bpn)
        b.done(lat)
        return r
    return run


_POROUS = {}


def porous_mask(b: Bench, dims):
    if dims not in _POROUS:
        _POROUS[dims] = b.workloads.porous_spheres(dims, (0, 1, 1), 6.0, 12.0, 0.2, b.workloads.SEED)[0]
    return _POROUS[dims]


def v_porous(general):
    def run(b: Bench):
        from paper_1801_04586_amd import Lattice

        np = b.np
        pdims = (640, 320, 320)
        mask = porous_mask(b, pdims)
        rates = nonslip_rates(b.workloads, 0.02) if general else b.workloads.rates(0.02)
        lat = Lattice(pdims, (0, 1, 1), "f32", rates, force=(2e-6, 0, 0), solid=mask, device=b.dev)
        lat.init()
        lat.step(3)
        pn = int(np.prod(pdims))
        fluid = int((mask == 0).sum())
        bpn = (2 * 27 * 4 * fluid + pn) / pn  # populations of fluid nodes + the solid mask
        ms = b.step_ms(lat)
        r = b.record(pn, ms, bpn, mflups_fluid=round(fluid / (ms * 1e-3) / 1e6, 1),
                     launch="two fused steps" if lat.uses_fused_pairs else "one step",
                     solid_fraction=round(1 - fluid / pn, 4))
        if general:
            r["rates"] = "s3 = (16 - 8 s2)/(8 - s2), s2b = s2"
        if lat.uses_fused_pairs:
            lat.set_fused_steps(False)
            r["single_step"] = b.record(pn, b.step_ms(lat), bpn)
        b.done(lat)
        return r
    return run


def v_adjoint_channel(b: Bench):
    """End-to-end gradient of the adjoint channel case: 64^3, T = 200, checkpoint every 20, FP32."""
    from paper_1801_04586_amd import Lattice
    from paper_1801_04586_amd.adjoint import flow_loss

    torch, np, wl = b.torch, b.np, b.workloads
    cdims, T, K = (64, 64, 64), 200, 20
    Fc = wl.gaussian_force(cdims, 1e-6, wl.SEED)
    lat = Lattice(cdims, (0, 1, 0), "f32", wl.rates(0.05), force_field=Fc, device=b.dev)
    lat.init()
    s0 = lat.state.clone()
    utc = torch.from_numpy(wl.channel_target(cdims, (0, 1, 0), 1e-4)).to(b.dev, torch.float32)
    Ft = torch.from_numpy(Fc).to(b.dev, torch.float32)
    st = torch.from_numpy(wl.rates(0.05))
    times = []
    for _ in range(3):
        Fr, sr = Ft.clone().requires_grad_(True), st.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        flow_loss(Fr, sr, lat, s0, utc, T, K).backward()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    cn = int(np.prod(cdims))
    tbest = min(times)
    b.done(lat)
    return {"gradient_seconds": round(tbest, 4), "node_updates_per_s_M": round(cn * T * 3 / tbest / 1e6, 1),
            "note": "forward T steps + recompute T steps + T adjoint steps, 64^3 (cache-resident, launch-bound)"}


def _adjoint_lattice(b: Bench, adims, storage="f32"):
    from paper_1801_04586_amd import Lattice

    wl = b.workloads
    mask = porous_mask(b, adims)
    Fa = wl.gaussian_force(adims, 1e-6, wl.SEED)
    lat = Lattice(adims, (0, 1, 1), storage, wl.rates(0.02), force=(2e-6, 0, 0), force_field=Fa, solid=mask,
                  device=b.dev)
    lat.init()
    lat.step(5)
    return lat, mask, Fa


def _adjoint_step_and_recompute(b: Bench, lat, K: int, keep: int):
    """Times of one adjoint step and of the recompute per step (clbm_trajectory keeping `keep` states, as
    the gradient recomputes a segment), in ms; and of one backward segment (recompute of K - 1 states
    plus K adjoint steps)."""
    torch = b.torch
    shape = lat.shape
    dt = lat.ctx.adjoint_dtype  # FP64 for FP64 storage, else FP32
    ut = torch.zeros((3,) + shape, dtype=dt, device=b.dev)
    lam = torch.empty((27,) + shape, dtype=dt, device=b.dev)
    lam2 = torch.empty_like(lam)
    gF = torch.zeros((3,) + shape, dtype=dt, device=b.dev)
    gs = torch.zeros(10, dtype=torch.float64, device=b.dev)
    lat.ctx.loss_seed(lat.state, ut, lam, gF, None)
    bufs = [lam, lam2]

    def adj10():
        for _ in range(5):
            lat.ctx.adjoint_step(lat.state, bufs[0], bufs[1], gF, gs)
            lat.ctx.adjoint_step(lat.state, bufs[1], bufs[0], gF, gs)

    adj10()
    adj_ms = b.ms(adj10, 10)
    states = [lat.new_state() for _ in range(keep)]
    lat.ctx.trajectory(lat.state, states)
    traj_ms = b.ms(lambda: lat.ctx.trajectory(lat.state, states), keep, reps=5)
    seg_ms = None
    if keep == K - 1:
        seg = [lat.state] + states

        def segment():
            lat.ctx.trajectory(seg[0], seg[1:])
            for t in range(K - 1, -1, -1):
                lat.ctx.adjoint_step(seg[t], bufs[t % 2], bufs[1 - t % 2], gF, gs)

        segment()
        seg_ms = b.ms(segment, 1, reps=5)
    del states
    return adj_ms, traj_ms, seg_ms


def v_adjoint_porous_crop_f64(b: Bench):
    """The adjoint step, its recompute and one backward segment (K = 20) on the same 256x128x128 crop with
    FP64 storage (FP64 adjoint populations and force gradient)."""
    np = b.np
    adims, K = (256, 128, 128), 20
    lat, mask, _ = _adjoint_lattice(b, adims, "f64")
    an = int(np.prod(adims))
    adj_ms, traj_ms, seg_ms = _adjoint_step_and_recompute(b, lat, K, K - 1)
    fl = float((mask == 0).mean())
    r = {"adjoint": b.record(an, adj_ms, ADJ_BYTES_F64,
                             frac_fluid=round(fl * ADJ_BYTES_F64 * an / (adj_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)),
         "recompute": b.record(an, traj_ms, bytes_per_node("f64", True, True), launch="clbm_trajectory (single steps)"),
         "backward_segment_K20": {"ms": round(seg_ms, 4), "adjoint_steps_per_s_M": round(an * K / (seg_ms * 1e-3) / 1e6, 1),
                                  "note": "recompute of 19 states + 20 adjoint steps, as the gradient runs it"},
         "solid_fraction": round(float(mask.mean()), 4)}
    b.done(lat)
    return r


def v_adjoint_porous_crop(b: Bench):
    """Adjoint step on the 256x128x128 crop of the porous duct (FP32, walls in y and z, spheres, per-node
    force field), the recompute the gradient runs (fused pairs that keep both states), one backward
    segment of K = 20, and the gradient of the flow loss end to end (T = 40, K = 20)."""
    from paper_1801_04586_amd.adjoint import flow_loss

    torch, np, wl = b.torch, b.np, b.workloads
    adims, K = (256, 128, 128), 20
    lat, mask, Fa = _adjoint_lattice(b, adims)
    an = int(np.prod(adims))
    adj_ms, traj_ms, seg_ms = _adjoint_step_and_recompute(b, lat, K, K - 1)
    fwd_bpn = bytes_per_node("f32", True, True)
    fl = float((mask == 0).mean())
    r = {"adjoint": b.record(an, adj_ms, ADJ_BYTES, frac_fluid=round(fl * ADJ_BYTES * an / (adj_ms * 1e-3) / 1e9
                                                                       / HBM_PEAK_GBS, 4)),
         "recompute": b.record(an, traj_ms, fwd_bpn, launch="clbm_trajectory (single steps)"),
         "backward_segment_K20": {"ms": round(seg_ms, 4), "adjoint_steps_per_s_M": round(an * K / (seg_ms * 1e-3) / 1e6, 1),
                                  "note": "recompute of 19 states + 20 adjoint steps, as the gradient runs it"},
         "solid_fraction": round(float(mask.mean()), 4)}
    Ta, Ka = 40, 20
    s0a = lat.state.clone()
    ut = torch.zeros((3,) + lat.shape, dtype=torch.float32, device=b.dev)
    Fta = torch.from_numpy(Fa).to(b.dev, torch.float32)
    sta = torch.from_numpy(wl.rates(0.02))
    times = []
    for _ in range(3):
        Fr, sr = Fta.clone().requires_grad_(True), sta.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        flow_loss(Fr, sr, lat, s0a, ut, Ta, Ka).backward()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    tg = min(times)
    r["gradient_T40_K20"] = {"seconds": round(tg, 4),
                             "node_updates_per_s_M": round(an * Ta * 3 / tg / 1e6, 1),
                             "note": "forward 40 steps + recompute + 40 adjoint steps"}
    b.done(lat)
    return r


def v_adjoint_porous_full(b: Bench):
    """The adjoint step and its recompute on the full 640x320x320 porous duct."""
    np = b.np
    adims = (640, 320, 320)
    lat, mask, _ = _adjoint_lattice(b, adims)
    an = int(np.prod(adims))
    adj_ms, traj_ms, _ = _adjoint_step_and_recompute(b, lat, 20, 4)
    fl = float((mask == 0).mean())
    r = {"adjoint": b.record(an, adj_ms, ADJ_BYTES, frac_fluid=round(fl * ADJ_BYTES * an / (adj_ms * 1e-3) / 1e9
                                                                       / HBM_PEAK_GBS, 4)),
         "recompute": b.record(an, traj_ms, bytes_per_node("f32", True, True), launch="clbm_trajectory, 4 states"),
         "adjoint_with_recompute_mlups": round(an / ((adj_ms + traj_ms) * 1e-3) / 1e6, 1),
         "solid_fraction": round(float(mask.mean()), 4)}
    b.done(lat)
    return r


VARIANTS = {
    "kolmogorov_512_f32_single": v_kolmogorov_single,
    "kolmogorov_512_f32_dense": v_kolmogorov_dense,
    "kolmogorov_512_f64": v_kolmogorov_storage("f64"),
    "kolmogorov_512_f16": v_kolmogorov_storage("f16"),
    "kolmogorov_512_bf16": v_kolmogorov_storage("bf16"),
    "kolmogorov_512_general_f32": v_kolmogorov_general,
    "kolmogorov_512_mrt_f32": v_kolmogorov_mrt,
    "kolmogorov_512_d3q19_f32": v_kolmogorov_d3q19("f32"),
    "kolmogorov_512_d3q19_f64": v_kolmogorov_d3q19("f64"),
    "kolmogorov_512_d3q19_f16": v_kolmogorov_d3q19("f16"),
    "cavity_256_cascaded_f32": v_cavity("cascaded"),
    "cavity_256_mrt_f32": v_cavity("mrt"),
    "cavity_256_cascaded_f64": v_cavity("cascaded", "f64"),
    "table_I_latency": v_table_I_latency,
    "table_I_bandwidth": v_table_I_bandwidth,
    "taylor_green_128_f64": v_taylor_green("f64"),
    "taylor_green_128_f32": v_taylor_green("f32"),
    "porous_640x320x320_f32": v_porous(False),
    "porous_640x320x320_general_f32": v_porous(True),
    "adjoint_channel_64_f32": v_adjoint_channel,
    "adjoint_porous_256x128x128_f32": v_adjoint_porous_crop,
    "adjoint_porous_256x128x128_f64": v_adjoint_porous_crop_f64,
    "adjoint_porous_640x320x320_f32": v_adjoint_porous_full,
}


# ------------------------------------------------------------------------------------------------ headline
def headline(b: Bench, args):
    torch = b.torch
    lat = b.kolmogorov_lattice()
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
    nodes = b.nodes
    mlups = nodes * args.steps / wall / 1e6
    bpn = bytes_per_node("f32", True, False)
    # algorithmic bytes of the node updates done in the timed region, per unit of kernel time
    achieved = bpn * nodes * args.steps / (event_ms * 1e-3) / 1e9
    log(f"[bench] f32 ({'two fused steps per launch' if fused else 'one step per launch'}): {ms_per_step:.3f} "
        f"ms/step wall, {kernel_ms:.3f} ms/launch, {mlups:.0f} MLUPS, {achieved:.0f} GB/s algorithmic")
    _, _, _, nbad = lat.moments(fields=False)
    if nbad:
        log(f"[bench] WARNING: {nbad} non-finite nodes")
    if args.copy_calibration:
        tmp = torch.empty_like(lat.state)
        for _ in range(5):
            lat.ctx.copy(lat.state, tmp)
        cms = b.ms(lambda: [lat.ctx.copy(lat.state, tmp) for _ in range(5)], 5, reps=3)
        log(f"[bench] copy {lat.state.numel() * 4 / 1e9:.2f} GB: {cms:.3f} ms = "
            f"{2 * lat.state.numel() * 4 / (cms * 1e-3) / 1e9:.0f} GB/s read+write")
        del tmp
    traffic = pmc_traffic(PMC_FUSED if fused else PMC_SINGLE, b.L, fused)
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
            "workload": f"kolmogorov_{b.L}^3",
            "nodes": nodes,
            "storage": "f32 deviations f - w",
            "force": "per-node FP32 field, F0 = 1e-5, k = 4",
            "nu": 0.005,
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
    step_ms = event_ms / args.steps
    b.done(lat)
    return result, b.record(nodes, step_ms, bpn, launch="two fused steps" if fused else "one step")


def accuracy(b: Bench):
    torch = b.torch
    steps = 500
    acc = {}
    l64 = b.kolmogorov_lattice("f64")
    l64.step(steps)
    _, u64, _, _ = l64.moments()
    b.done(l64)
    nrm = torch.linalg.vector_norm(u64).item()
    umax = u64.abs().max().item()
    for storage in ("f32", "f16", "bf16"):
        ls = b.kolmogorov_lattice(storage)
        ls.step(steps)
        _, us, _, nb = ls.moments()
        d = us - u64
        acc[storage] = {"l2_rel": float(torch.linalg.vector_norm(d).item() / nrm),
                        "max_rel": float(d.abs().max().item() / umax), "nonfinite": int(nb)}
        log(f"[bench] accuracy {storage} after {steps} steps: {acc[storage]}")
        b.done(ls)
        del us, d
    acc["reference"] = f"FP64 storage, same inputs, {steps} steps; u_max = {umax:.4e}"
    acc["targets"] = "FP32: L2-relative below 1e-5 (its max-relative error is stated beside it)"
    del u64
    return acc


def cpu_baseline(b: Bench, args):
    import oracle

    np, wl = b.np, b.workloads
    _, _, F, u0 = b.kolmogorov()
    dims, L = b.dims, b.L
    wd = (128, 128, 32)
    g = oracle.Geometry(dims, (0, 0, 0), (0, 0, 0), wd)
    sl = (slice(0, wd[2]), slice(0, wd[1]), slice(0, wd[0]))
    rates = wl.rates(0.005)
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
    res = {"value": round(wn * nsteps / tc / 1e6, 4), "unit": "MLUPS", "cores": oracle.num_threads(),
           "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "sample": f"{wd[0]}x{wd[1]}x{wd[2]} window of the {L}^3 Kolmogorov lattice, {nsteps} steps, FP64 dense "
                     f"27x27 oracle, {tc:.1f} s"}
    budget = args.cpu_seconds / 2

    def timed_run(geom, f, rates_, max_steps, full=False, **kw):
        # one step to size the run, then as many as fit the budget (at most max_steps; all of them if full)
        t0 = time.perf_counter()
        f = oracle.step(geom, f, rates_, **kw)
        t1 = time.perf_counter() - t0
        n = max_steps if full else max(1, min(max_steps, int(budget / max(t1, 1e-4))))
        t0 = time.perf_counter()
        for _ in range(n):
            f = oracle.step(geom, f, rates_, **kw)
        dt = time.perf_counter() - t0
        return geom.n * n / dt / 1e6, n, dt

    nthreads = oracle.num_threads()
    oracle.set_num_threads(1)
    w1 = (64, 64, 16)
    g1 = oracle.Geometry(dims, (0, 0, 0), (0, 0, 0), w1)
    s1 = (slice(0, w1[2]), slice(0, w1[1]), slice(0, w1[0]))
    f1 = oracle.init(g1, None, np.ascontiguousarray(u0[(slice(None),) + s1]))
    m1, n1, d1 = timed_run(g1, f1, rates, 50, force_field=np.ascontiguousarray(F[(slice(None),) + s1]))
    oracle.set_num_threads(nthreads)
    res["single_core"] = {"value": round(m1, 4), "cores": 1,
                          "sample": f"{w1[0]}x{w1[1]}x{w1[2]} window of the same lattice, {n1} steps, {d1:.1f} s"}
    pc = wl.POISEUILLE
    gp = oracle.Geometry(pc.dims, pc.walls)
    # the 16x32x16 channel in full (3000 steps, a few seconds)
    mp, npo, dp_ = timed_run(gp, oracle.init(gp), pc.rates(), pc.steps, full=True, force=pc.force_uniform)
    tc2 = wl.TGV128
    gt = oracle.Geometry(tc2.dims, tc2.walls)
    rt0, ut0 = wl.taylor_green_3d(tc2.dims, 0.04)
    mt, ntg, dtg = timed_run(gt, oracle.init(gt, rt0, ut0), tc2.rates(), tc2.steps)
    res["other_workloads"] = {
        pc.name: {"value": round(mp, 4), "steps": npo, "of_steps": pc.steps, "seconds": round(dp_, 2)},
        tc2.name: {"value": round(mt, 4), "steps": ntg, "of_steps": tc2.steps, "seconds": round(dtg, 2)},
        "note": "the channel in full; the Taylor-Green vortex as many steps as fit the time budget"}
    log(f"[bench] cpu baseline: {res}")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--size", type=int, default=512, help="edge of the cubic Kolmogorov lattice")
    ap.add_argument("--only", default="", help="comma-separated variant names (or 'headline'); no headline line. "
                    "Variants: " + ", ".join(VARIANTS))
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
    only = [s for s in args.only.split(",") if s]
    unknown = [s for s in only if s not in VARIANTS and s != "headline"]
    if unknown:
        print(f"unknown variants {unknown}; known: headline, {', '.join(VARIANTS)}", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    b = Bench(args)
    log(f"[bench] Kolmogorov {b.dims}, nu=0.005; kernel source {kernel_sha()}")

    if only:
        out = {"only": only, "variants": {}}
        for name in only:
            if name == "headline":
                out["headline"], _ = headline(b, args)
                continue
            log(f"[bench] {name}")
            out["variants"][name] = VARIANTS[name](b)
            log(f"[bench] {name}: {out['variants'][name]}")
        print(json.dumps(out), flush=True)
        return

    result, head_rec = headline(b, args)
    if not args.primary_only:
        variants = {HEADLINE: head_rec}
        if not args.no_variants:
            for name, fn in VARIANTS.items():
                log(f"[bench] {name}")
                variants[name] = fn(b)
                log(f"[bench] {name}: {variants[name]}")
            result["speedup_f32_over_f64"] = round(variants["kolmogorov_512_f64"]["ms_per_step"] /
                                                   head_rec["ms_per_step"], 3)
        result["variants"] = variants
        if not args.no_accuracy:
            result["accuracy_vs_f64"] = accuracy(b)
    if not args.no_cpu and not args.primary_only:
        result["cpu_baseline"] = cpu_baseline(b, args)
    result["context"] = {
        "paper_cpu": "0.45 MLUPS: C++ CLBM, i7-6500U laptop, 5x101x5 shear wave (Table I), context only",
        "paper_table_I_seconds": {"5x101x5": [56.028, 26.042, 2.151], "5x201x5": [111.838, 51.728, 2.162],
                                  "5x401x5": [217.027, 101.179, 2.145], "columns": "t_C, t_S, t_C/t_S (CPU)"},
        "hbm_peak_gbs": HBM_PEAK_GBS,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
