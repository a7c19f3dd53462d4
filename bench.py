"""Benchmark: time to a 1e-10 true residual, mixed precision vs plain FP64 CG, and Dslash HBM GB/s.

    python bench.py [--steps K] [--warmup W] [--workload 5] [--prec f16] [--no-cpu-baseline]

The default line is the largest single-GPU workload: a 48^3x144 lattice with 8 right-hand sides,
m = 0.0062, solved to true residual 1e-10.  A step is one pass of the whole hot path over the
workload's synthetic input, which is resident in HBM before timing starts: pack the links (phases,
boundary signs and c_N folded; FP64 + FP16) and solve (4m^2 - D_eo D_oe) x = b for all 8 right-hand
sides with mixed-precision CG (FP16 storage, FP32 arithmetic, FP64 reliable updates), 8 right-hand
sides per Dslash launch.  The two Dslash launches of every 10th iteration are bracketed by HIP events
on the solver's stream; their average duration gives the roofline figure.

Beside the timed steps the line carries, each with its own timing:
  * the plain FP64 CG of the same system (warm-up, then timed solves);
  * `paper_lattice`: the 28^3x96 single-RHS record (FP16 and FP32 mixed precision, FP64 CG);
  * `with_network`: the same 8-RHS solve with the learned preconditioner in flexible CG (the network
    trained on 24^3x48 pairs and applied on the large lattice);
  * `stream_ceiling`: a read-only streaming kernel of the library on this GPU;
  * `cpu_baseline`: the oracle on the host, one thread and all threads, extrapolated from a bounded
    sample of the same workload;
  * `leg_seconds`: the wall time of every leg.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-10 true residual vs plain FP64 CG; Dslash HBM GB/s (% of peak)"
HBM_PEAK_GBPS = 8000.0
# Compulsory bytes per output site and right-hand side of one Dslash launch:
# 16 links + link scales + input and output colour vectors; the xpay launch of the
# solver also reads d at the output site.  f16 colour vectors are 12 B of codes + a 4 B scale.
LINK = {"f64": 144, "f32": 72, "f16": 36}
LINK12 = {"f64": 96, "f32": 48, "f16": 24}   # three-hop link stored as two rows (12 real parameters)
LSCALE = {"f64": 0, "f32": 0, "f16": 8}
VEC = {"f64": 48, "f32": 24, "f16": 16}
FLOPS_PER_SITE = 1146


def link_bytes_per_site(prec: str, long12: bool) -> int:
    return 8 * LINK[prec] + 8 * (LINK12[prec] if long12 else LINK[prec]) + LSCALE[prec]


def dslash_bytes_per_site(prec: str, xpay: bool = False, long12: bool = True) -> int:
    return link_bytes_per_site(prec, long12) + 2 * VEC[prec] + (VEC[prec] if xpay else 0)


def launch_bytes(prec: str, half: int, nrhs: int, long12: bool = True) -> float:
    """Compulsory bytes of one Dslash launch of the solver, the plain and the xpay launch averaged:
    each link once, every RHS's input and output vectors, half a vector more for the xpay read of d."""
    return half * (link_bytes_per_site(prec, long12) + nrhs * 2.5 * VEC[prec])


def host_info():
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model or platform.processor()}


def cpu_workers() -> int:
    """Threads for the oracle's threaded mode: the cores this process may run on, at most 16 (the host
    share that goes with one GPU of a node)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(fat, lng, b, dims, mass, iters_fp64, nrhs=1, workers=None):
    """The oracle as it stands on a bounded sample of the workload: one operator application
    M = 4m^2 - D_eo D_oe on one right-hand side of the full lattice (the bulk of a CG iteration: the
    iteration adds a few vector updates), timed with BLAS pinned to one thread (`oracle.dslash.apply_m`)
    and, if workers > 1, with the chunked operator on that many threads (`apply_m_chunked`).  Each is
    scaled to a whole solve: per-application time x the GPU FP64 iteration count x nrhs."""
    from threadpoolctl import threadpool_limits

    from oracle.dslash import apply_m, apply_m_chunked

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        apply_m(fat, lng, b, dims, mass)
        dt1 = time.perf_counter() - t0
    out = {"value": dt1 * iters_fp64 * nrhs, "unit": "s", "cores": 1, "kind": "oracle",
           "sample": f"one operator application (oracle.dslash.apply_m, 1 thread) on one RHS of "
                     f"{'x'.join(map(str, dims))} took {dt1:.2f} s; scaled by the GPU FP64 iteration count "
                     f"{iters_fp64} and {nrhs} RHS (extrapolated)",
           "per_iteration_s": dt1}
    if workers and workers > 1:
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            apply_m_chunked(fat, lng, b, dims, mass, workers=workers)
            dtn = time.perf_counter() - t0
        out["threaded"] = {"value": dtn * iters_fp64 * nrhs, "unit": "s", "cores": workers,
                           "per_iteration_s": dtn,
                           "sample": f"the chunked oracle operator (apply_m_chunked) on {workers} threads, "
                                     f"same sample and scaling"}
    return out


def stream_ceiling(torch, nbytes=4 << 30, reps=10):
    """Read-only streaming kernel of the library (stag_stream_read) over a 4 GiB buffer: the HBM read
    ceiling on this GPU, with HIP events on the stream the kernel runs on."""
    from paper_1010_4782_amd._lib import check, lib

    buf = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    sink = torch.empty(nbytes // 32768, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()

    def run():
        check(lib().stag_stream_read(buf.data_ptr(), nbytes, sink.data_ptr(), int(s.cuda_stream)),
              "stag_stream_read")

    run()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        run()
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del buf, sink
    return {"GBps": nbytes / (ms * 1e-3) / 1e9, "frac_of_hbm_peak": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "bytes_read": nbytes, "avg_launch_us": ms * 1e3, "kernel": "k_stream_read (stag_stream_read)"}


def long12_for(a, prec: str, nrhs_all) -> bool:
    """Three-hop link storage of a leg: two rows (12 reals, the third rebuilt in the kernel) or all 18.
    auto: 18 reals for a mixed-precision leg whose lattices all have a multiple of 8 RHS, where a lane can
    then take 8 RHS and the rebuild's arithmetic costs more than its 96 saved bytes per site (measured:
    8-RHS FP16 launch at 48^3x144, 1630 us with 18 reals and 8 RHS per lane against 1841 us with 12 reals,
    whose rebuild only fits 4 per lane); 12 reals otherwise (FP64, and fewer RHS per lane: bound by bytes)."""
    if a.long_links == "12":
        return True
    if a.long_links == "18":
        return False
    nrhs_all = [nrhs_all] if isinstance(nrhs_all, int) else list(nrhs_all)
    return prec == "f64" or any(n % 8 for n in nrhs_all)


def measured_traffic(prec: str, dims, long_su3: bool, nrhs: int = 1, shape=None):
    """HBM bytes per Dslash launch from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source, this workload, this long-link storage and this launch shape; otherwise None."""
    import hashlib

    tag = f"dslash_{prec}_{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]}" + (f"_{nrhs}rhs" if nrhs > 1 else "")
    path = os.path.join(ROOT, "profiles", f"{tag}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec["source_files"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    # traffic per long-link storage and launch shape: "l12:wg,rhs_per_lane,lds_stage,tile_order,t_chunks"
    if shape is None:
        return None
    key = ("l12:" if long_su3 else "l18:") + ",".join(
        str(shape[k]) for k in ("wg", "rhs_per_lane", "lds_stage", "tile_order", "t_chunks"))
    return rec["traffic_bytes_per_launch"].get(key)


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


class Solves:
    """One workload's lattices, links and sources resident on the GPU, and its timed solves."""

    def __init__(self, wid, a, keep_host=False):
        import torch

        from paper_1010_4782_amd.stagcg import Lattice
        from stag_inputs import WORKLOADS, workload_links_device, workload_sources

        self.w = WORKLOADS[wid]
        self.wid = wid
        self.a = a
        self.tol = self.w["tol"]
        self.rel_int = self.w.get("reliable_interval", 50)
        self.probs, self.host = [], []
        for li, (dims, nrhs) in enumerate(self.w["lattices"]):
            fat, lng = workload_links_device(wid, li)
            b = workload_sources(wid, li)
            lat = Lattice(dims)
            self.probs.append(dict(lat=lat, dims=dims, nrhs=nrhs, fat=fat, lng=lng, b=torch.from_numpy(b).cuda()))
            self.host.append(b if keep_host else None)
        torch.cuda.synchronize()

    def long12(self, prec):
        return long12_for(self.a, prec, [p["nrhs"] for p in self.probs])

    def host_links(self, li=0):
        return self.probs[li]["fat"].cpu().numpy(), self.probs[li]["lng"].cpu().numpy()

    def step(self, prec, profile=10, precs=None):
        """load_links on every lattice, then one batched solve per mass; returns (infos, solve seconds)."""
        import torch

        from paper_1010_4782_amd.stagcg import cg_solve_batch

        precs = precs or ("f64", prec)
        for p in self.probs:
            p["lat"].load_links(p["fat"], p["lng"], -1.0 / 24.0, precs=precs, long_su3=self.long12(prec))
            if self.a.shape and prec != "f64":
                p["lat"].set_dslash_shape(prec, p["nrhs"], *self.a.shape)
        torch.cuda.synchronize()  # load_links is asynchronous; keep its packing out of solve_s
        infos, t_solve = [], 0.0
        for m in self.w["masses"]:
            batch = [(p["lat"], p["b"], [m] * p["nrhs"], None) for p in self.probs]
            t0 = time.perf_counter()
            _, inf = cg_solve_batch(batch, tol=self.tol, prec=prec, reliable_interval=self.rel_int, profile=profile,
                                    max_iter=self.a.max_iter, max_restarts=0 if self.a.max_iter else 5,
                                    raise_on_fail=self.a.max_iter == 0, autotune=not self.a.no_autotune)
            t_solve += time.perf_counter() - t0  # the call synchronises before returning
            infos.append(inf)
        return infos, t_solve

    def timed(self, prec, steps, warmup, precs=None):
        import torch

        for i in range(warmup):
            self.step(prec, precs=precs)
            log(f"{self.w['name']} {prec}: warmup {i} done")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        all_infos, solve = [], 0.0
        for i in range(steps):
            infos, ts = self.step(prec, precs=precs)
            all_infos.append(infos)
            solve += ts
            its = [max(x["iters"] for x in inf) for inf in infos]
            res = max(x["true_resid"] for inf in infos for x in inf)
            log(f"{self.w['name']} {prec}: step {i}: iterations {its}, worst true resid {res:.3e}")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        return all_infos, elapsed / steps, solve / steps

    def dslash_rate(self, infos, prec):
        """Algorithmic GB/s of the inner-iteration Dslash launches (plain and xpay averaged), from the
        sampled HIP-event timings of the solves."""
        flat = [inf for infos_ in infos for inf in infos_]
        ms = sum(i[0]["dslash_ms"] for i in flat)
        calls = sum(i[0]["dslash_calls"] for i in flat)
        per_launch = sum(launch_bytes(prec, p["lat"].half, p["nrhs"], self.long12(prec)) for p in self.probs)
        avg = ms / max(calls, 1)
        sites = sum(p["lat"].half * p["nrhs"] for p in self.probs)
        return dict(GBps=per_launch / (avg * 1e-3) / 1e9, avg_launch_us=avg * 1e3, bytes_per_launch=per_launch,
                    launches=calls, gflops=sites * FLOPS_PER_SITE / (avg * 1e-3) / 1e9)

    def summary(self, infos):
        last = infos[-1]
        return {"iters": [max(x["iters"] for x in inf) for inf in last],
                "reliable_updates": [max(x["n_reliable"] for x in inf) for inf in last],
                "true_resid": max(x["true_resid"] for inf in last for x in inf),
                "dslash_shape": {"wg": last[0][0]["dslash_wg"], "rhs_per_lane": last[0][0]["dslash_rhs"],
                                 "lds_stage": last[0][0]["dslash_lds"], "tile_order": last[0][0]["dslash_order"],
                                 "t_chunks": last[0][0]["dslash_chunks"]}}

    def shape_name(self):
        return "+".join(f"{p['dims'][0]}^3x{p['dims'][3]}x{p['nrhs']}" if p["dims"][0] == p["dims"][2] else
                        f"{'x'.join(map(str, p['dims']))}x{p['nrhs']}" for p in self.probs)

    def close(self):
        import torch

        for p in self.probs:
            p["lat"].close()
        self.probs = []
        torch.cuda.synchronize()
        torch.cuda.empty_cache()


def solve_record(s: Solves, a, steps, warmup, fp64_steps, extra_precs=()):
    """Mixed precision timed over the steps, plain FP64 CG over fp64_steps (after one warm-up), and any
    further inner precisions timed like the first.  Returns (record, infos of the mixed-precision steps)."""
    infos, per_step, solve = s.timed(a.prec, steps, warmup)
    rate = s.dslash_rate(infos, a.prec)
    rec = {"step_s": per_step, "solve_s": solve, **{"mp_" + k: v for k, v in s.summary(infos).items()},
           "dslash_" + a.prec: {**rate, "frac_of_hbm_peak": rate["GBps"] / HBM_PEAK_GBPS}}
    for prec in extra_precs:
        inf2, step2, solve2 = s.timed(prec, steps, 1, precs=("f64", prec))
        r2 = s.dslash_rate(inf2, prec)
        rec["mixed_" + prec] = {"step_s": step2, "solve_s": solve2, **s.summary(inf2),
                                "dslash": {**r2, "frac_of_hbm_peak": r2["GBps"] / HBM_PEAK_GBPS}}
    if fp64_steps > 0:
        i64, step64, solve64 = s.timed("f64", fp64_steps, 1, precs=("f64",))
        r64 = s.dslash_rate(i64, "f64")
        rec["fp64_cg"] = {"step_s": step64, "solve_s": solve64, "timed_solves": fp64_steps, **s.summary(i64),
                          "dslash": {**r64, "frac_of_hbm_peak": r64["GBps"] / HBM_PEAK_GBPS}}
        rec["speedup_vs_fp64_cg"] = step64 / per_step
        rec["speedup_solve_only"] = solve64 / solve
        log(f"{s.w['name']} fp64 CG: {rec['fp64_cg']['iters']} it, {step64:.3f} s per solve")
    return rec, infos


def break_even_stall(mp_solve_s, mp_iters, t_net_s, tol, window=1):
    """Stall-test parameters under which flexible CG with the network has to keep pace with the
    mixed-precision CG it would hand over to: a window of `window` FCG iterations (each about one
    mixed-precision iteration of operator and vector work plus one network application on every RHS)
    must cut ||r|| at least as much as the mixed-precision solve does in the same time at its average
    rate (||r|| / ||b|| from 1 to tol in mp_solve_s).  Returns (stall_window, stall_ratio)."""
    t_it = mp_solve_s / max(1, mp_iters) + t_net_s
    return window, tol ** (window * t_it / mp_solve_s)


def run_learned_preconditioner(a):
    """Workload 4: train the network on (b, x = M^-1 b) pairs made by the batched FP64 solver, then time
    flexible CG with it against plain FP64 CG and mixed-precision CG on the workload's source."""
    import torch

    from paper_1010_4782_amd.stagcg import Lattice, Net
    from stag_inputs import WORKLOADS, gaussian_source_device, workload_links, workload_sources

    w = WORKLOADS[4]
    dims, _ = w["lattices"][0]
    mass, tol = w["masses"][0], w["tol"]
    npairs = a.train_pairs if a.train_pairs > 0 else w["train_pairs"]
    fat, lng = workload_links(4)
    b_eval = torch.from_numpy(workload_sources(4)).cuda()
    lat = Lattice(dims)
    lat.load_links(torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda(), -1.0 / 24.0,
                   precs=("f64", "f32", a.prec), long_su3=long12_for(a, a.prec, 1))
    del fat, lng
    half = lat.half
    chunk = 8
    bs = torch.empty((npairs, half, 3), dtype=torch.complex128, device="cuda")
    xs = torch.empty_like(bs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c0 in range(0, npairs, chunk):
        n = min(chunk, npairs - c0)
        bs[c0:c0 + n] = gaussian_source_device(dims, 4000 + c0, n)
        x, _ = lat.cg_solve(bs[c0:c0 + n].contiguous(), mass, tol=tol, prec=a.prec, autotune=True)
        xs[c0:c0 + n] = x
        if (c0 // chunk) % 25 == 0:
            log(f"training data {c0 + n}/{npairs}")
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = Net(lat, layers=w["layers"], channels=w["channels"], seed=1, hermitian=True)
    t0 = time.perf_counter()
    tinfo = net.train(bs, xs, epochs=a.epochs, batch=8, lr=a.lr, loss=a.loss, mass=mass)
    t_train = time.perf_counter() - t0
    log(f"trained: loss {tinfo['loss_first']:.4f} -> {tinfo['loss_last']:.4f} in {t_train:.1f} s")
    del bs, xs
    res = {}

    def run(name, kw):
        lat.cg_solve(b_eval, mass, tol=tol, autotune=True, **kw)  # warm-up (and tuning)
        times = []
        for _ in range(max(1, a.steps)):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, info = lat.cg_solve(b_eval, mass, tol=tol, **kw)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
        res[name] = {"s": sum(times) / len(times), "iters": info[0]["iters"], "true_resid": info[0]["true_resid"],
                     "fell_back": info[0]["fell_back"], "n_reliable": info[0]["n_reliable"]}
        log(f"{name}: {res[name]}")

    run("fp64_cg", {})
    run("mixed_" + a.prec, dict(prec=a.prec))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(20):
        net.apply(b_eval)
    torch.cuda.synchronize()
    t_apply = (time.perf_counter() - t1) / 20
    mp = res["mixed_" + a.prec]
    win, ratio = break_even_stall(mp["s"], mp["iters"], t_apply, tol, a.stall_window)
    run("fcg_net_" + a.prec, dict(net=net, stall_window=win, stall_ratio=ratio, prec=a.prec))
    res["fcg_net_" + a.prec]["stall_window"], res["fcg_net_" + a.prec]["stall_ratio"] = win, ratio
    fcg = res["fcg_net_" + a.prec]
    out = {"metric": METRIC, "value": fcg["s"], "unit": "s", "n_gpus": 1, "steps": a.steps, "warmup": 1,
           "ms_per_step": 1e3 * fcg["s"], "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 (network f32; FP64 reliable updates)", "data": "synthetic",
           "config": {"workload": f"{dims[0]}^3x{dims[3]}, m={mass}, flexible CG with a {w['layers']}-layer, "
                                  f"{w['channels']}-channel gauge-covariant network vs plain CG, true residual {tol}",
                      "train_pairs": npairs, "epochs": a.epochs, "loss": a.loss},
           "solves": res, "speedup_fcg_vs_fp64_cg": res["fp64_cg"]["s"] / fcg["s"],
           "speedup_fcg_vs_mixed": res["mixed_" + a.prec]["s"] / fcg["s"],
           "network_apply_ms": 1e3 * t_apply, "training": {"data_s": t_data, "train_s": t_train, **tinfo}}
    saved = res["fp64_cg"]["s"] - fcg["s"]
    out["break_even_solves"] = (t_data + t_train) / saved if saved > 0 else None
    print(json.dumps(out), flush=True)
    return 0


def fattening_leg(dims, reps=2):
    """stag_fatten_links on the workload's lattice: asqtad one-hop links and three-hop products of a thin
    SU(3) field drawn on the GPU (the links of the solves are drawn directly, as the recipe says; this times
    the step that would make them from a gauge configuration)."""
    import torch

    from paper_1010_4782_amd.stagcg import Lattice
    from stag_inputs import random_su3_field_device

    U = random_su3_field_device(dims, 77)
    lat = Lattice(dims)
    fat, lng = torch.empty_like(U), torch.empty_like(U)
    lat.fatten_links(U, 1.0, fat, lng)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        lat.fatten_links(U, 1.0, fat, lng)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    sites = dims[0] * dims[1] * dims[2] * dims[3]
    lat.close()
    del U, fat, lng
    return {"lattice": list(dims), "ms": ms, "sites_per_s": sites / (ms * 1e-3),
            "recipe": "asqtad (1, 3, 5, 7-link staples and Lepage paths), u0 = 1, FP64; long = U U U"}


def network_leg(a, s: Solves, mass, tol, rel_int, mp_s, mp_iters, fp64_s):
    """The third change on the large workload: mixed precision, multi-RHS and the learned preconditioner
    together.  The network is trained on the 24^3x48 lattice (links drawn by the same recipe) at this
    workload's mass, then its weights (the layers are gauge-covariant stencils with site-independent
    channel weights, so they do not depend on the volume) are loaded into a network on the large
    lattice.  The solve is flexible CG with the network on all RHS, which hands each RHS to the
    mixed-precision CG when its residual stalls; the stall test asks it to keep pace with the
    mixed-precision CG measured before (break_even_stall)."""
    import torch

    from paper_1010_4782_amd.stagcg import Lattice, Net
    from stag_inputs import WORKLOADS, gaussian_source_device, workload_links

    w4 = WORKLOADS[4]
    dims4, _ = w4["lattices"][0]
    npairs = a.train_pairs if a.train_pairs > 0 else 256
    fat, lng = workload_links(4)
    small = Lattice(dims4)
    small.load_links(torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda(), -1.0 / 24.0,
                     precs=("f64", "f32", a.prec), long_su3=long12_for(a, a.prec, 8))
    del fat, lng
    bs = torch.empty((npairs, small.half, 3), dtype=torch.complex128, device="cuda")
    xs = torch.empty_like(bs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c0 in range(0, npairs, 8):
        n = min(8, npairs - c0)
        bs[c0:c0 + n] = gaussian_source_device(dims4, 5000 + c0, n)
        xs[c0:c0 + n], _ = small.cg_solve(bs[c0:c0 + n].contiguous(), mass, tol=tol, prec=a.prec,
                                          reliable_interval=rel_int, autotune=True)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net_s = Net(small, layers=w4["layers"], channels=w4["channels"], seed=1, hermitian=True)
    t0 = time.perf_counter()
    tinfo = net_s.train(bs, xs, epochs=a.epochs, batch=8, lr=a.lr, loss=a.loss, mass=mass)
    t_train = time.perf_counter() - t0
    log(f"network trained on {dims4}: loss {tinfo['loss_first']:.4f} -> {tinfo['loss_last']:.4f} "
        f"({npairs} pairs, {t_data:.1f} s data, {t_train:.1f} s training)")
    weights = net_s.get_weights()
    del bs, xs, net_s
    small.close()
    p = s.probs[0]
    lat = p["lat"]
    lat.load_links(p["fat"], p["lng"], -1.0 / 24.0, precs=("f64", "f32", a.prec), long_su3=s.long12(a.prec))
    net = Net(lat, layers=w4["layers"], channels=w4["channels"], seed=1, hermitian=True)
    net.set_weights(weights)
    net.apply(p["b"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    net.apply(p["b"])
    torch.cuda.synchronize()
    t_apply = time.perf_counter() - t1
    win, ratio = break_even_stall(mp_s, mp_iters, t_apply, tol, a.stall_window)
    kw = dict(tol=tol, prec=a.prec, reliable_interval=rel_int, net=net, stall_window=win, stall_ratio=ratio,
              autotune=True)
    lat.cg_solve(p["b"], mass, **kw)  # warm-up
    times = []
    for _ in range(max(1, a.network_solves)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, info = lat.cg_solve(p["b"], mass, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
    t_solve = sum(times) / len(times)
    net.close()
    res = {"solve_s": t_solve, "solve_s_min_max": [min(times), max(times)], "timed_solves": len(times),
           "iters": max(i["iters"] for i in info), "fell_back": sum(i["fell_back"] for i in info),
           "true_resid": max(i["true_resid"] for i in info), "network_apply_ms_all_rhs": 1e3 * t_apply,
           "stall_window": win, "stall_ratio": ratio,
           "speedup_vs_mixed_only": mp_s / t_solve, "speedup_vs_fp64_cg": (fp64_s / t_solve) if fp64_s else None,
           "training": {"lattice": list(dims4), "pairs": npairs, "epochs": a.epochs, "data_s": t_data,
                        "train_s": t_train, "loss_first": tinfo["loss_first"], "loss_last": tinfo["loss_last"]}}
    log(f"network + mixed precision: {res['iters']} it, {t_solve:.3f} s, {res['fell_back']} RHS fell back")
    return res


def run_shard_demo(a):
    """One GPU's share of a t-decomposed Dslash (the design of a multi-GPU run, exercised on one GPU):
    P slabs of Lt/P slices, each with its two 3-slice faces copied in from its neighbours; the slab
    Dslash of every slab must equal the unsplit Dslash bit for bit.  Times the unsplit launch, one slab
    launch and one face copy (device to device on this GPU), all FP64, with HIP events."""
    import torch

    from paper_1010_4782_amd.stagcg import Lattice
    from stag_inputs import WORKLOADS, workload_links_device, workload_sources

    w = WORKLOADS[a.workload]
    dims, nrhs = w["lattices"][0]
    P = a.shard_demo
    Lt = dims[3]
    if Lt % P or (Lt // P) % 2:
        print(f"--shard-demo {P}: Lt = {Lt} must split into P slabs of an even number of slices", file=sys.stderr)
        return 2
    lt = Lt // P
    fat, lng = workload_links_device(a.workload)
    b = torch.from_numpy(workload_sources(a.workload)).cuda()
    lat = Lattice(dims)
    lat.load_links(fat, lng, -1.0 / 24.0, precs=("f64",), long_su3=long12_for(a, "f64", 1))
    del fat, lng
    S = lat.half // Lt
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn, reps=10):
        fn()
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3  # us

    par = 1
    ref = lat.dslash(b, par)
    ok = True
    ext = torch.empty((nrhs, (lt + 6) * S, 3), dtype=torch.complex128, device="cuda")
    for k in range(P):
        t0 = k * lt
        lo, hi = ((t0 - 3) % Lt) * S, ((t0 + lt) % Lt) * S
        ext[:, 3 * S:(lt + 3) * S] = b[:, t0 * S:(t0 + lt) * S]          # own slices
        ext[:, :3 * S] = b[:, lo:lo + 3 * S]                              # face from slab k-1
        ext[:, (lt + 3) * S:] = b[:, hi:hi + 3 * S]                        # face from slab k+1
        out = lat.dslash_slab(ext, par, t0, lt)
        ok &= bool(torch.equal(out, ref[:, t0 * S:(t0 + lt) * S]))
    face = b[:, :3 * S].contiguous()
    recv = torch.empty_like(face)
    us_full = timed(lambda: lat.dslash(b, par, out=ref))
    out = torch.empty((nrhs, lt * S, 3), dtype=torch.complex128, device="cuda")
    us_slab = timed(lambda: lat.dslash_slab(ext, par, 0, lt, out=out))
    us_face = timed(lambda: recv.copy_(face))
    face_bytes = face.numel() * 16
    res = {"metric": "shard demo: slab Dslash on one GPU's share, loopback exchange", "workload": w["name"],
           "dims": list(dims), "nrhs": nrhs, "slabs": P, "slab_dims": [dims[0], dims[1], dims[2], lt],
           "loopback_bitwise_equal": ok, "dslash_f64_unsplit_us": us_full, "dslash_f64_slab_us": us_slab,
           "slab_over_unsplit": us_slab / us_full, "face_bytes_per_direction": face_bytes,
           "face_copy_device_us": us_face,
           "face_over_xgmi_link_us_estimate": face_bytes / 153e9 * 1e6,
           "note": "xGMI time is face bytes / 153 GB/s (one link), an estimate: no second GPU here"}
    print(json.dumps(res), flush=True)
    return 0 if ok else 1


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=5, choices=[1, 2, 3, 4, 5, 6])
    ap.add_argument("--prec", default="f16", choices=["f32", "f16"])
    ap.add_argument("--fp64-steps", type=int, default=-1,
                    help="timed plain FP64 CG solves after one warm-up (default: 2 on 48^3x144, 5 otherwise; 0 skips)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison solves")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the workload's own solves: no 28^3x96 record, network leg or stream ceiling")
    ap.add_argument("--max-iter", type=int, default=0,
                    help="cap the inner iterations (for counter-collection runs; the solve then stops early)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default launch shape instead of timing the candidates (for "
                         "counter-collection runs, where every dispatch is serialised and timings mean nothing)")
    ap.add_argument("--long-links", default="auto", choices=["auto", "12", "18"],
                    help="three-hop link storage: two rows (12 reals, third rebuilt) or all 18; auto: 18 for a "
                         "mixed-precision leg whose lattices all have a multiple of 8 RHS, else 12")
    ap.add_argument("--no-long-su3", action="store_true", help="same as --long-links 18")
    ap.add_argument("--shape", type=lambda v: [int(x) for x in v.split(",")], default=None,
                    metavar="WG,R,LDS,ORDER,CHUNKS",
                    help="pin the mixed-precision Dslash launch shape (for counter runs without the tuner)")
    ap.add_argument("--train-pairs", type=int, default=0,
                    help="workloads 4 and 5: training pairs (0: 2000 for workload 4, 256 for workload 5)")
    ap.add_argument("--epochs", type=int, default=5, help="workloads 4 and 5: training epochs")
    ap.add_argument("--network-solves", type=int, default=2,
                    help="workload 5: timed solves of the network leg after one warm-up (mean reported)")
    ap.add_argument("--stall-window", type=int, default=1,
                    help="workloads 4 and 5: flexible-CG iterations per stall test (break-even ratio scaled to it)")
    ap.add_argument("--lr", type=float, default=2e-3, help="workloads 4 and 5: Adam step size")
    ap.add_argument("--loss", default="residual", choices=["residual", "solution"],
                    help="workloads 4 and 5: training loss")
    ap.add_argument("--no-net", action="store_true", help="workload 5: skip the leg with the learned preconditioner")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="end with one 1 GiB device-to-device copy, the known-size kernel that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters of a rocprofv3 run")
    ap.add_argument("--shard-demo", type=int, default=0, metavar="P",
                    help="instead of the solve: split the workload's first lattice into P time slabs (one per GPU "
                         "of a multi-GPU run), exchange the 3-slice faces on this one GPU, apply the slab Dslash, "
                         "check the assembled result against the unsplit one and time both")
    a = ap.parse_args(argv)
    if a.no_long_su3:
        a.long_links = "18"
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X; multi-GPU runs are not supported.",
              file=sys.stderr)
        return 2

    if a.workload == 4:
        return run_learned_preconditioner(a)
    if a.shard_demo:
        return run_shard_demo(a)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    legs = {}
    t_leg = time.perf_counter()
    s = Solves(a.workload, a)
    legs["inputs"] = time.perf_counter() - t_leg
    log(f"inputs for {s.w['name']} in {legs['inputs']:.1f} s")
    big = a.workload == 5
    fp64_steps = 0 if a.no_fp64 else (a.fp64_steps if a.fp64_steps >= 0 else (2 if big else 5))
    t_leg = time.perf_counter()
    rec, infos = solve_record(s, a, a.steps, a.warmup, 0)
    legs["mixed_precision"] = time.perf_counter() - t_leg
    t_leg = time.perf_counter()
    if fp64_steps:
        i64, step64, solve64 = s.timed("f64", fp64_steps, 1, precs=("f64",))
        r64 = s.dslash_rate(i64, "f64")
        fp64 = {"step_s": step64, "solve_s": solve64, "timed_solves": fp64_steps, **s.summary(i64),
                "dslash": {**r64, "frac_of_hbm_peak": r64["GBps"] / HBM_PEAK_GBPS}}
        legs["fp64_cg"] = time.perf_counter() - t_leg
        log(f"fp64 CG: {fp64['iters']} it, {step64:.3f} s per solve")
    else:
        fp64 = None
    rate = rec["dslash_" + a.prec]
    d0, n0 = s.probs[0]["dims"], s.probs[0]["nrhs"]
    traffic = (measured_traffic(a.prec, d0, s.long12(a.prec), n0, rec["mp_dslash_shape"])
               if len(s.probs) == 1 else None)
    out = {
        "metric": METRIC, "value": rec["step_s"], "unit": "s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * rec["step_s"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "storage": a.prec, "data": "synthetic",
        "config": {"workload": f"{s.shape_name()} (lattice x RHS), m={s.w['masses']}, fat (0.6 SU(3) + noise) and "
                               f"Naik links, true residual {s.tol}",
                   "lattices": [list(p["dims"]) for p in s.probs], "nrhs": [p["nrhs"] for p in s.probs],
                   "masses": s.w["masses"], "tol": s.tol,
                   "solver": f"mixed-precision CG, {a.prec} storage, FP64 reliable update every {s.rel_int} "
                             f"iterations or after a 10x residual drop, all RHS of a lattice in each launch",
                   "step": "load_links + solve",
                   "long_links": {leg: ("12 reals (two rows, third rebuilt)" if s.long12(pr) else "18 reals")
                                  for leg, pr in (("mixed_precision", a.prec), ("fp64_cg", "f64"))}},
        "solve_s": rec["solve_s"],
        "mp_iters": rec["mp_iters"], "mp_reliable_updates": rec["mp_reliable_updates"],
        "mp_true_resid": rec["mp_true_resid"], "dslash_shape": rec["mp_dslash_shape"],
        "roofline": {"bound": "hbm", "achieved": rate["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": rate["GBps"] / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": f"k_dslash<{a.prec}>, {n0} RHS per launch (plain and xpay launches)",
                     "avg_launch_us": rate["avg_launch_us"], "launches": rate["launches"],
                     "bytes_per_launch": rate["bytes_per_launch"]},
        "dslash_" + a.prec: rate,
    }
    if fp64:
        out["fp64_cg"] = fp64
        out["fp64_cg_s"] = fp64["step_s"]
        out["speedup_vs_fp64_cg"] = fp64["step_s"] / rec["step_s"]
        out["speedup_solve_only"] = fp64["solve_s"] / rec["solve_s"]
    host = b_host = None
    if (big or a.workload == 2) and not a.no_cpu_baseline:
        # host copies for the oracle, taken before the network leg reloads the links
        host = s.host_links()
        b_host = s.probs[0]["b"][0].cpu().numpy()
    if big and not a.no_extras:
        if not a.no_net:
            t_leg = time.perf_counter()
            out["with_network"] = network_leg(a, s, s.w["masses"][0], s.tol, s.rel_int, rec["solve_s"],
                                              max(rec["mp_iters"]), fp64["solve_s"] if fp64 else None)
            legs["with_network"] = time.perf_counter() - t_leg
        s.close()
        t_leg = time.perf_counter()
        s2 = Solves(2, a)
        pl, _ = solve_record(s2, a, a.steps, a.warmup, 5, extra_precs=("f32",) if a.prec == "f16" else ())
        pl["workload"] = f"{s2.shape_name()}, m={s2.w['masses']}"
        pl["traffic"] = measured_traffic(a.prec, s2.probs[0]["dims"], s2.long12(a.prec), s2.probs[0]["nrhs"],
                                         pl["mp_dslash_shape"])
        out["paper_lattice"] = pl
        s2.close()
        legs["paper_lattice"] = time.perf_counter() - t_leg
        t_leg = time.perf_counter()
        out["stream_ceiling"] = stream_ceiling(torch)
        legs["stream_ceiling"] = time.perf_counter() - t_leg
    if big and not a.no_extras:
        t_leg = time.perf_counter()
        out["link_fattening"] = fattening_leg(s.w["lattices"][0][0])
        legs["link_fattening"] = time.perf_counter() - t_leg
    if a.calibration_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB device to device")
        del src, dst
    if host is not None:
        log("cpu baseline (oracle) ...")
        t_leg = time.perf_counter()
        iters = (fp64["iters"] if fp64 else rec["mp_iters"])[0]
        cb = cpu_baseline(host[0], host[1], b_host, s.w["lattices"][0][0], s.w["masses"][0], iters,
                          nrhs=s.w["lattices"][0][1], workers=cpu_workers())
        cb["host"] = host_info()
        out["cpu_baseline"] = cb
        legs["cpu_baseline"] = time.perf_counter() - t_leg
    out["leg_seconds"] = legs
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
