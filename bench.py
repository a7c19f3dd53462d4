"""Benchmark: time to a 1e-10 true residual on 28^3 x 96, mixed precision vs plain FP64 CG, plus Dslash GB/s.

    python bench.py [--steps K] [--warmup W] [--workload 2] [--prec f16] [--no-cpu-baseline]

A step is one pass of the whole hot path over the workload's synthetic input,
which is resident in HBM before timing starts: pack the links (phases, signs and
c_N folded; FP64 + the inner precision) and solve (4m^2 - D_eo D_oe) x = b with
mixed-precision CG and FP64 reliable updates to true residual 1e-10.  The plain
FP64 CG solve of the same system is timed once beside it.  The two Dslash launches
of every 10th CG iteration of the timed steps are bracketed by HIP events on the
solver's stream; their average duration gives the roofline figure.  Prints one JSON
line.
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


def cpu_baseline(fat, lng, b, dims, mass, iters_fp64):
    """The oracle's CG as it stands, on one core, for a bounded sample: one Fig. 1 iteration
    (plus the initial and final residual) on the full lattice, scaled to a whole solve."""
    import numpy as np

    from oracle.cg import cg
    from oracle.dslash import apply_m

    # pin every BLAS / OpenMP pool numpy may use to one thread, so that "cores" is what ran
    from threadpoolctl import threadpool_limits

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        cg(lambda v: apply_m(fat, lng, v, dims, mass), b, tol=1e-10, max_iter=1, max_restarts=0)
        dt = time.perf_counter() - t0
    per_iter = dt / 3.0   # three operator applications: r = b - A x, one iteration, the true residual
    return {"value": per_iter * iters_fp64, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"one oracle CG iteration on {dims[0]}^3x{dims[3]} ({dt:.1f} s for 3 operator "
                      f"applications), scaled by the GPU FP64 iteration count {iters_fp64}; extrapolated",
            "per_iteration_s": per_iter}


def copy_ceiling(torch, nbytes=2 << 30, reps=10):
    """Device-to-device copy of a 2 GiB buffer: the streaming ceiling on this GPU (read + write bytes / time)."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        dst.copy_(src)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del src, dst
    return {"GBps": 2 * nbytes / (ms * 1e-3) / 1e9, "bytes_read": nbytes, "bytes_written": nbytes,
            "avg_launch_us": ms * 1e3}


def measured_traffic(prec: str, dims, long_su3: bool):
    """HBM bytes per Dslash launch from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source, this workload and this long-link storage; otherwise None."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"dslash_{prec}_{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("long_su3", False) != long_su3:
        return None
    h = hashlib.sha256()
    for f in rec["source_files"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def run_learned_preconditioner(a, out_json):
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
                   precs=("f64", "f32", a.prec), long_su3=not a.no_long_su3)
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
        x, _ = lat.cg_solve(bs[c0:c0 + n].contiguous(), mass, tol=tol, autotune=True)
        xs[c0:c0 + n] = x
        if (c0 // chunk) % 25 == 0:
            print(f"# training data {c0 + n}/{npairs}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = Net(lat, layers=w["layers"], channels=w["channels"], seed=1, hermitian=True)
    t0 = time.perf_counter()
    tinfo = net.train(bs, xs, epochs=a.epochs, batch=8, lr=a.lr, loss=a.loss, mass=mass)
    t_train = time.perf_counter() - t0
    print(f"# trained: loss {tinfo['loss_first']:.4f} -> {tinfo['loss_last']:.4f} in {t_train:.1f} s",
          file=sys.stderr, flush=True)
    del bs, xs
    res = {}
    for name, kw in (("fcg_net", dict(net=net, stall_window=10)), ("fp64_cg", {}),
                     ("mixed_" + a.prec, dict(prec=a.prec))):
        lat.cg_solve(b_eval, mass, tol=tol, autotune=True, **kw)  # warm-up (and tuning)
        times = []
        for _ in range(max(1, a.steps)):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, info = lat.cg_solve(b_eval, mass, tol=tol, **kw)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
        res[name] = {"s": min(times), "iters": info[0]["iters"], "true_resid": info[0]["true_resid"],
                     "fell_back": info[0]["fell_back"]}
        print(f"# {name}: {res[name]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(20):
        net.apply(b_eval)
    torch.cuda.synchronize()
    t_apply = (time.perf_counter() - t1) / 20
    out = {"metric": METRIC, "value": res["fcg_net"]["s"], "unit": "s", "n_gpus": 1, "steps": a.steps, "warmup": 1,
           "ms_per_step": 1e3 * res["fcg_net"]["s"], "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64 (network f32)", "data": "synthetic",
           "config": {"workload": f"{dims[0]}^3x{dims[3]}, m={mass}, flexible CG with a {w['layers']}-layer, "
                                  f"{w['channels']}-channel gauge-covariant network vs plain CG, true residual {tol}",
                      "train_pairs": npairs, "epochs": a.epochs, "loss": a.loss},
           "solves": res, "speedup_fcg_vs_fp64_cg": res["fp64_cg"]["s"] / res["fcg_net"]["s"],
           "network_apply_ms": 1e3 * t_apply, "training": {"data_s": t_data, "train_s": t_train, **tinfo}}
    saved = res["fp64_cg"]["s"] - res["fcg_net"]["s"]
    out["break_even_solves"] = (t_data + t_train) / saved if saved > 0 else None
    print(json.dumps(out), flush=True)
    return 0


def network_leg(a, p, mass, tol, rel_int, mp_s, fp64_s):
    """Workload 5's third leg: mixed precision, multi-RHS and the learned preconditioner together.  The
    network is trained on the workload-4 lattice (24^3x48, links drawn by the same recipe) at this
    workload's mass, then its weights (which do not depend on the volume: the layers are gauge-covariant
    stencils with site-independent channel weights) are loaded into a network on the large lattice.  The
    solve is flexible CG with the network on all RHS, which hands each RHS to the mixed-precision CG when
    its residual stalls."""
    import torch

    from paper_1010_4782_amd.stagcg import Lattice, Net
    from stag_inputs import WORKLOADS, gaussian_source_device, workload_links

    w4 = WORKLOADS[4]
    dims4, _ = w4["lattices"][0]
    npairs = a.train_pairs if a.train_pairs > 0 else 256
    fat, lng = workload_links(4)
    small = Lattice(dims4)
    small.load_links(torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda(), -1.0 / 24.0,
                     precs=("f64", "f32", a.prec), long_su3=not a.no_long_su3)
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
    print(f"# network trained on {dims4}: loss {tinfo['loss_first']:.4f} -> {tinfo['loss_last']:.4f} "
          f"({npairs} pairs, {t_data:.1f} s data, {t_train:.1f} s training)", file=sys.stderr, flush=True)
    weights = net_s.get_weights()
    del bs, xs, net_s, small
    lat = p["lat"]
    lat.load_links(p["fat"], p["lng"], -1.0 / 24.0, precs=("f64", "f32", a.prec), long_su3=not a.no_long_su3)
    net = Net(lat, layers=w4["layers"], channels=w4["channels"], seed=1, hermitian=True)
    net.set_weights(weights)
    kw = dict(tol=tol, prec=a.prec, reliable_interval=rel_int, net=net, stall_window=10, autotune=True)
    lat.cg_solve(p["b"], mass, **kw)  # warm-up
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, info = lat.cg_solve(p["b"], mass, **kw)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    net.apply(p["b"][:1].contiguous())
    torch.cuda.synchronize()
    t_apply = time.perf_counter() - t1
    res = {"solve_s": t_solve, "iters": max(i["iters"] for i in info), "fell_back": sum(i["fell_back"] for i in info),
           "true_resid": max(i["true_resid"] for i in info), "network_apply_ms_per_rhs": 1e3 * t_apply,
           "speedup_vs_mixed_only": mp_s / t_solve, "speedup_vs_fp64_cg": (fp64_s / t_solve) if fp64_s else None,
           "training": {"lattice": list(dims4), "pairs": npairs, "epochs": a.epochs, "data_s": t_data,
                        "train_s": t_train, "loss_first": tinfo["loss_first"], "loss_last": tinfo["loss_last"]}}
    print(f"# network + mixed precision: {res['iters']} it, {t_solve:.3f} s, {res['fell_back']} RHS fell back",
          file=sys.stderr, flush=True)
    return res


def run_shard_demo(a):
    """One GPU's share of a t-decomposed Dslash (the design of a multi-GPU run, exercised on one GPU):
    P slabs of Lt/P slices, each with its two 3-slice faces copied in from its neighbours; the slab
    Dslash of every slab must equal the unsplit Dslash bit for bit.  Times the unsplit launch, one slab
    launch and one face copy (device to device on this GPU), all FP64, with HIP events."""
    import torch

    from paper_1010_4782_amd.stagcg import Lattice
    from stag_inputs import WORKLOADS, workload_links, workload_sources

    w = WORKLOADS[a.workload]
    dims, nrhs = w["lattices"][0]
    P = a.shard_demo
    Lt = dims[3]
    if Lt % P or (Lt // P) % 2:
        print(f"--shard-demo {P}: Lt = {Lt} must split into P slabs of an even number of slices", file=sys.stderr)
        return 2
    lt = Lt // P
    fat, lng = workload_links(a.workload)
    b = torch.from_numpy(workload_sources(a.workload)).cuda()
    lat = Lattice(dims)
    lat.load_links(torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda(), -1.0 / 24.0, precs=("f64",),
                   long_su3=not a.no_long_su3)
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
    ap.add_argument("--workload", type=int, default=2, choices=[1, 2, 3, 4, 5, 6])
    ap.add_argument("--prec", default="f16", choices=["f32", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison solve")
    ap.add_argument("--max-iter", type=int, default=0,
                    help="cap the inner iterations (for counter-collection runs; the solve then stops early)")
    ap.add_argument("--profile-every", type=int, default=10,
                    help="bracket the Dslash launches of every k-th CG iteration with HIP events (each event "
                         "record idles the GPU for a few us, so timing every iteration would slow the solve)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default launch shape instead of timing the candidates (for "
                         "counter-collection runs, where every dispatch is serialised and timings mean nothing)")
    ap.add_argument("--no-long-su3", action="store_true",
                    help="store the three-hop links with all 18 reals instead of two rows (12 parameters)")
    ap.add_argument("--train-pairs", type=int, default=0,
                    help="workloads 4 and 5: training pairs (0: 2000 for workload 4, 256 for workload 5)")
    ap.add_argument("--epochs", type=int, default=5, help="workloads 4 and 5: training epochs")
    ap.add_argument("--lr", type=float, default=2e-3, help="workloads 4 and 5: Adam step size")
    ap.add_argument("--loss", default="residual", choices=["residual", "solution"],
                    help="workloads 4 and 5: training loss")
    ap.add_argument("--no-net", action="store_true",
                    help="workload 5: skip the leg that adds the learned preconditioner")
    ap.add_argument("--shard-demo", type=int, default=0, metavar="P",
                    help="instead of the solve: split the workload's first lattice into P time slabs (one per GPU "
                         "of a multi-GPU run), exchange the 3-slice faces on this one GPU, apply the slab Dslash, "
                         "check the assembled result against the unsplit one and time both")
    a = ap.parse_args(argv)
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X; multi-GPU runs are not supported.",
              file=sys.stderr)
        return 2

    if a.workload == 4:
        return run_learned_preconditioner(a, None)
    if a.shard_demo:
        return run_shard_demo(a)

    import numpy as np
    import torch

    from paper_1010_4782_amd.stagcg import Lattice, cg_solve_batch
    from stag_inputs import WORKLOADS, workload_links, workload_sources

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    w = WORKLOADS[a.workload]
    tol = w["tol"]
    rel_int = w.get("reliable_interval", 50)
    t_gen = time.perf_counter()
    dev = torch.device("cuda:0")
    host, probs = [], []
    for li, (dims, nrhs) in enumerate(w["lattices"]):
        fat, lng = workload_links(a.workload, li)
        b = workload_sources(a.workload, li)
        lat = Lattice(dims)
        probs.append(dict(lat=lat, dims=dims, nrhs=nrhs, fat=torch.from_numpy(fat).to(dev),
                          lng=torch.from_numpy(lng).to(dev), b=torch.from_numpy(b).to(dev)))
        host.append((fat, lng, b))
        if a.workload != 2:
            del fat, lng
            host[-1] = None
    print(f"# inputs generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    masses = w["masses"]
    precs = ("f64", a.prec)

    def step(prec, profile=None):
        """load_links on every lattice, then one batched solve per mass; returns the infos."""
        profile = a.profile_every if profile is None else profile
        for p in probs:
            p["lat"].load_links(p["fat"], p["lng"], -1.0 / 24.0, precs=precs, long_su3=not a.no_long_su3)
        torch.cuda.synchronize()  # load_links is asynchronous; keep its packing out of solve_s
        infos = []
        for m in masses:
            batch = [(p["lat"], p["b"], [m] * p["nrhs"], None) for p in probs]
            t_s = time.perf_counter()
            xs, inf = cg_solve_batch(batch, tol=tol, prec=prec, reliable_interval=rel_int, profile=profile,
                                     max_iter=a.max_iter, max_restarts=0 if a.max_iter else 5,
                                     raise_on_fail=a.max_iter == 0, autotune=not a.no_autotune)
            solve_time[0] += time.perf_counter() - t_s  # the call synchronises before returning
            infos.append(inf)
            if "source_sites" in w:  # propagators: the pion correlator of every source is part of the step
                corr.append((probs[0]["lat"].pion_correlator(xs[0], m), xs[0]))
        return infos

    corr = []

    solve_time = [0.0]

    def dslash_rate(infos, prec):
        """Algorithmic GB/s of the inner-iteration Dslash launches (plain and xpay averaged).  The bytes
        are the compulsory ones of the whole batch: each lattice's links once per launch, whatever the
        launch shape (a shape with fewer RHS per lane than the lattice has re-reads them: that is not
        counted), plus every RHS's input and output vectors (and half a vector for the xpay read)."""
        ms = sum(i[0]["dslash_ms"] for i in infos)
        calls = sum(i[0]["dslash_calls"] for i in infos)
        per_launch = 0.0
        for p in probs:
            site = link_bytes_per_site(prec, not a.no_long_su3) + p["nrhs"] * 2.5 * VEC[prec]
            per_launch += p["lat"].half * site
        avg = ms / max(calls, 1)
        sites = sum(p["lat"].half * p["nrhs"] for p in probs)
        return per_launch / (avg * 1e-3) / 1e9, avg, per_launch, calls, sites * FLOPS_PER_SITE / (avg * 1e-3) / 1e9

    def paper_count_rate(prec, avg_ms):
        """GB/s under the paper's own count (Sec. 2): every link, every one of the 16 neighbour colour
        vectors and the output counted per site, no cache reuse; single RHS only."""
        site = link_bytes_per_site(prec, not a.no_long_su3) + 17 * VEC[prec]
        return sum(p["lat"].half for p in probs) * site / (avg_ms * 1e-3) / 1e9

    for i in range(a.warmup):
        step(a.prec)
        print(f"# warmup {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    solve_time[0] = 0.0
    t0 = time.perf_counter()
    all_infos = []
    for i in range(a.steps):
        infos = step(a.prec)
        all_infos.append(infos)
        its = [max(x["iters"] for x in inf) for inf in infos]
        res = max(x["true_resid"] for inf in infos for x in inf)
        print(f"# step {i}: max iterations per batch {its}, worst true resid {res:.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    mp_corr = corr[-1] if corr else None  # the last timed mixed-precision step's correlator
    ms_per_step = 1e3 * elapsed / a.steps
    flat = [inf for infos in all_infos for inf in infos]
    achieved, avg_ms, bytes_per_launch, d_calls, gflops = dslash_rate(flat, a.prec)
    last = all_infos[-1]
    d0 = probs[0]["dims"]
    shape = "+".join(f"{p['dims'][0]}^3x{p['dims'][3]}x{p['nrhs']}" if p["dims"][0] == p["dims"][2] else
                     f"{'x'.join(map(str, p['dims']))}x{p['nrhs']}" for p in probs)
    out = {
        "metric": METRIC, "value": ms_per_step / 1e3, "unit": "s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "storage": a.prec, "data": "synthetic",
        "config": {"workload": f"{shape} (lattice x RHS), m={masses}, fat (0.6 SU(3) + noise) and Naik links, "
                               f"true residual {tol}", "lattices": [list(p["dims"]) for p in probs],
                   "nrhs": [p["nrhs"] for p in probs], "masses": masses, "tol": tol,
                   "solver": f"mixed-precision CG, {a.prec} storage, FP64 reliable update every {rel_int} "
                             f"iterations or after a 10x residual drop", "step": "load_links + solve",
                   "long_links": "18 reals" if a.no_long_su3 else "12 reals (two rows, third rebuilt)"},
        "solve_s": solve_time[0] / a.steps,
        "mp_iters": [max(x["iters"] for x in inf) for inf in last],
        "mp_reliable_updates": [max(x["n_reliable"] for x in inf) for inf in last],
        "mp_true_resid": max(x["true_resid"] for inf in last for x in inf),
        "dslash_shape": {"wg": last[0][0]["dslash_wg"], "rhs_per_lane": last[0][0]["dslash_rhs"],
                         "lds_stage": last[0][0]["dslash_lds"], "tile_order": last[0][0]["dslash_order"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": measured_traffic(a.prec, d0, not a.no_long_su3) if len(probs) == 1 and probs[0]["nrhs"] == 1 else None,
                     "kernel": f"k_dslash<{a.prec}> (plain and xpay launches)",
                     "avg_launch_us": avg_ms * 1e3, "launches": d_calls, "bytes_per_launch": bytes_per_launch},
    }
    if not a.no_fp64:
        torch.cuda.synchronize()
        solve_time[0] = 0.0
        t1 = time.perf_counter()
        i64 = step("f64")
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        gbs64, avg64, _, _, gf64 = dslash_rate(i64, "f64")
        out["fp64_cg_s"] = t64
        out["fp64_solve_s"] = solve_time[0]
        out["speedup_solve_only"] = solve_time[0] / out["solve_s"]
        out["fp64_iters"] = [max(x["iters"] for x in inf) for inf in i64]
        out["fp64_true_resid"] = max(x["true_resid"] for inf in i64 for x in inf)
        out["speedup_vs_fp64_cg"] = t64 / (ms_per_step / 1e3)
        out["dslash_f64"] = {"GBps": gbs64, "frac_of_hbm_peak": gbs64 / HBM_PEAK_GBPS, "avg_launch_us": avg64 * 1e3,
                             "gflops": gf64, "shape": {"wg": i64[0][0]["dslash_wg"], "rhs_per_lane": i64[0][0]["dslash_rhs"],
                                                       "lds_stage": i64[0][0]["dslash_lds"],
                                                       "tile_order": i64[0][0]["dslash_order"]}}
        print(f"# fp64 CG: {out['fp64_iters']} it, {t64:.3f} s, Dslash {gbs64:.0f} GB/s", file=sys.stderr, flush=True)
    out["dslash_" + a.prec] = {"GBps": achieved, "frac_of_hbm_peak": achieved / HBM_PEAK_GBPS,
                               "avg_launch_us": avg_ms * 1e3, "gflops": gflops}
    if all(p["nrhs"] == 1 for p in probs):
        out["dslash_" + a.prec]["GBps_paper_count"] = paper_count_rate(a.prec, avg_ms)
    if a.workload == 5 and not a.no_net:
        out["with_network"] = network_leg(a, probs[0], masses[0], tol, rel_int, out["solve_s"],
                                          out.get("fp64_solve_s"))
    if mp_corr is not None:
        C, x0 = mp_corr
        torch.cuda.synchronize()
        Ch = C.cpu().numpy()
        d0 = probs[0]["dims"]
        diag = []
        for s_, (sx, sy, sz, st) in enumerate(w["source_sites"]):
            cb = (sx + d0[0] * (sy + d0[1] * (sz + d0[2] * st))) // 2
            diag.append(sum(float(x0[3 * s_ + c, cb, c].real) for c in range(3)))
        out["propagators"] = {
            "sources": w["source_sites"], "correlator_t0_to_8": [list(map(float, row[:8])) for row in Ch],
            "sum_rule_rel_err": max(abs(Ch[s_].sum() - diag[s_]) / diag[s_] for s_ in range(len(diag))),
            "note": "C(t) = sum over time slice t of |G|^2, G_e = 2m chi, G_o = -D_oe chi; the sum over t equals "
                    "sum_c chi^(c)(x0)_c"}
    out["copy_ceiling"] = copy_ceiling(torch)
    if not a.no_cpu_baseline and a.workload == 2:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        iters = out.get("fp64_iters", out["mp_iters"])[0]
        fat, lng, b = host[0]
        cb = cpu_baseline(fat, lng, b[0], probs[0]["dims"], masses[0], iters)
        cb["host"] = host_info()
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
