"""Benchmark-size solves checked by the oracle: the GPU's solution x of every right-hand side goes back to
the host and the oracle recomputes its true residual ||b - M x|| / ||b|| (paper Fig. 1; the true-residual
rule of Sec. 2) with its own operator, chunked over sites and threaded so that 48^3x144 fits the time.

Sizes re-checked here: 28^3x96 (FP16 and FP32 mixed precision, plain FP64), the batched 16^4x4 +
24^3x48x12 + 32^3x64x8 workload at each of its three masses (every RHS), 48^3x144 with 8 right-hand sides
(every RHS, plus sampled Dslash sites in the launch shapes the solver uses: FP64 against the exact
operator, FP16 against the operator on identically rounded links and inputs within its rounding bound).
"""
import os

import numpy as np
import pytest
import torch

from oracle.cg import true_residuals
from oracle import lowprec
from oracle.dslash import apply_m_chunked, dslash_at_sites

pytestmark = pytest.mark.gpu

NAIK = -1.0 / 24.0
WORKERS = max(1, min(16, os.cpu_count() or 1))


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_resid(fat, lng, dims, b, x, masses):
    b = b.reshape((-1,) + b.shape[-2:])
    x = x.reshape(b.shape)
    return true_residuals(lambda v: apply_m_chunked(fat, lng, v, dims, masses, workers=WORKERS), b, x)


def check_solution(infos, resid, tol):
    """Every RHS converged, the oracle's residual is within the tolerance (5% for rounding of M x at
    these sizes) and agrees with the library's own FP64 recomputation."""
    for i, (info, r) in enumerate(zip(infos, resid)):
        print(f"   rhs {i}: iters {info['iters']} library {info['true_resid']:.4e} oracle {r:.4e}", flush=True)
        assert info["converged"] == 1
        assert r <= 1.05 * tol
        assert abs(r - info["true_resid"]) <= 0.02 * info["true_resid"]


@pytest.fixture(scope="module")
def c2():
    from paper_1010_4782_amd.stagcg import Lattice
    from stag_inputs import WORKLOADS, workload_links, workload_sources

    w = WORKLOADS[2]
    dims = w["lattices"][0][0]
    print(f"28^3x96 inputs ({dims})", flush=True)
    fat, lng = workload_links(2)
    b = workload_sources(2)
    lat = Lattice(dims)
    lat.load_links(torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda(), NAIK, precs=("f64", "f32", "f16"),
                   long_su3=True)
    yield dict(lat=lat, fat=fat, lng=lng, b=b, bt=torch.from_numpy(b).cuda(), dims=dims, mass=w["masses"][0],
               tol=w["tol"])
    lat.close()


@pytest.mark.parametrize("prec", ["f16", "f32", "f64"])
def test_paper_lattice_solve_checked_by_oracle(gpu_lib, c2, prec):
    """28^3x96, m = 0.0062: mixed precision (FP16 or FP32 storage, FP64 reliable updates every 50
    iterations) and plain FP64 CG, each to true residual 1e-10 as the oracle recomputes it."""
    print(f"28^3x96 solve {prec}", flush=True)
    x, info = c2["lat"].cg_solve(c2["bt"], c2["mass"], tol=c2["tol"], prec=prec, reliable_interval=50,
                                 autotune=True)
    r = oracle_resid(c2["fat"], c2["lng"], c2["dims"], c2["b"], x.cpu().numpy(), c2["mass"])
    check_solution(info, r, c2["tol"])


def test_point_source_fp16_solve_28cubed_96(gpu_lib, c2):
    """28^3x96, m = 0.0062, a point source in FP16 mixed precision: around iterations 12-14 the smallest
    site scales of r and d fall to 1e-39 (binary32 subnormals; the FP64 oracle CG shows the same), and the
    solve still converges to the true residual, which the oracle recomputes."""
    from stag_inputs import point_sources

    print("28^3x96 point-source f16 solve", flush=True)
    b = point_sources(c2["dims"], [(3, 5, 7, 11)])
    x, info = c2["lat"].cg_solve(torch.from_numpy(b).cuda(), c2["mass"], tol=c2["tol"], prec="f16",
                                 reliable_interval=50)
    r = oracle_resid(c2["fat"], c2["lng"], c2["dims"], b, x.cpu().numpy(), c2["mass"])
    check_solution(info, r, c2["tol"])


@pytest.mark.parametrize("mass", [0.01, 0.02, 0.05])
def test_batched_uneven_lattices_every_rhs_checked_by_oracle(gpu_lib, mass):
    """The batched workload at full size, one batch per mass: 16^4 x 4 + 24^3x48 x 12 + 32^3x64 x 8
    right-hand sides in one launch per stage, FP16 mixed precision with the autotuner, 12-real long
    links; the oracle re-checks all 24 solutions."""
    from paper_1010_4782_amd.stagcg import Lattice, cg_solve_batch
    from stag_inputs import WORKLOADS, workload_links, workload_sources

    w = WORKLOADS[3]
    print(f"batched full size, m = {mass}", flush=True)
    probs, hosts = [], []
    for li, (dims, nrhs) in enumerate(w["lattices"]):
        fat, lng = workload_links(3, li)
        b = workload_sources(3, li)
        lat = Lattice(dims)
        lat.load_links(torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda(), NAIK, precs=("f64", "f16"),
                       long_su3=True)
        probs.append((lat, torch.from_numpy(b).cuda(), [mass] * nrhs, None))
        hosts.append((fat, lng, dims, b))
    xs, infos = cg_solve_batch(probs, tol=w["tol"], prec="f16", autotune=True)
    k = 0
    for (fat, lng, dims, b), x in zip(hosts, xs):
        n = b.shape[0]
        print(f"  {dims} x {n}", flush=True)
        check_solution(infos[k:k + n], oracle_resid(fat, lng, dims, b, x.cpu().numpy(), mass), w["tol"])
        k += n


@pytest.fixture(scope="module")
def c5():
    """48^3x144 with 8 right-hand sides: links drawn on the GPU (the same tensors the oracle reads back)."""
    from paper_1010_4782_amd.stagcg import Lattice
    from stag_inputs import WORKLOADS, workload_links_device, workload_sources

    w = WORKLOADS[5]
    dims, nrhs = w["lattices"][0]
    print(f"48^3x144 inputs ({dims} x {nrhs} RHS)", flush=True)
    fat_d, lng_d = workload_links_device(5)
    lat = Lattice(dims)
    lat.load_links(fat_d, lng_d, NAIK, precs=("f64", "f16"), long_su3=True)
    fat, lng = fat_d.cpu().numpy(), lng_d.cpu().numpy()
    del fat_d, lng_d
    b = workload_sources(5)
    yield dict(lat=lat, fat=fat, lng=lng, b=b, bt=torch.from_numpy(b).cuda(), dims=dims, nrhs=nrhs,
               mass=w["masses"][0], tol=w["tol"])
    lat.close()


def test_large_lattice_dslash_sampled(gpu_lib, c5):
    """48^3x144 x 8 RHS in the solver's launch shapes (8 right-hand sides per lane; XCD-block order;
    LDS staging) against the oracle at sampled sites of every RHS, both output parities, FP64."""
    lat, fat, lng, b, bt, dims, nrhs = (c5[k] for k in ("lat", "fat", "lng", "b", "bt", "dims", "nrhs"))
    print("48^3x144 sampled dslash", flush=True)
    half = b.shape[1]
    rng = np.random.default_rng(5)
    sample = np.concatenate([rng.integers(0, half, 96), np.arange(32), np.arange(half - 32, half)])
    lat.set_dslash_shape("f64", nrhs, 64, 8)
    for par in (0, 1):
        out = lat.dslash(bt, par).cpu().numpy()
        ref = dslash_at_sites(fat, lng, b, dims, par, sample)
        for r in range(nrhs):
            assert rel(out[r][sample], ref[r]) <= 1e-12, (par, r)
    for shape in ((64, 4, 1), (64, 4, 0, 1), (128, 8, 0, 1)):
        lat.set_dslash_shape("f64", nrhs, *shape)
        assert np.array_equal(lat.dslash(bt, 1).cpu().numpy(), out), shape
    lat.set_dslash_shape("f64", nrhs, 0, 1)


def test_large_lattice_solve_every_rhs_checked_by_oracle(gpu_lib, c5):
    """48^3x144, m = 0.0062, 8 right-hand sides: FP16 mixed precision with multi-RHS launches, in the
    headline benchmark's configuration (three-hop links with all 18 reals, tuned launch shape); the oracle
    recomputes all 8 true residuals."""
    print("48^3x144 x 8 mixed-precision solve", flush=True)
    lat = c5["lat"]
    lat.load_links(torch.from_numpy(c5["fat"]).cuda(), torch.from_numpy(c5["lng"]).cuda(), NAIK,
                   precs=("f64", "f16"), long_su3=False)
    torch.cuda.empty_cache()
    x, info = lat.cg_solve(c5["bt"], c5["mass"], tol=c5["tol"], prec="f16", reliable_interval=50, autotune=True)
    print(f"   launch shape wg {info[0]['dslash_wg']} rhs/lane {info[0]['dslash_rhs']} order {info[0]['dslash_order']}",
          flush=True)
    print("   oracle residuals (chunked, threaded)", flush=True)
    r = oracle_resid(c5["fat"], c5["lng"], c5["dims"], c5["b"], x.cpu().numpy(), c5["mass"])
    check_solution(info, r, c5["tol"])


def _f16_sampled_check(lat, fat, lng, b, bt, dims, sample, long12):
    """FP16 Dslash at the sampled output sites of every RHS, both parities, within the rounding bound of
    the low-precision model (the operator in FP64 on the identically rounded links and inputs: FP32
    products over 48 complex terms, FP32 third-row rebuild for 12-real links, binary16 output rounding)."""
    u32 = 2.0 ** -24
    c = 300 if long12 else 200
    outs = []
    for par in (0, 1):
        out = lat.dslash(bt, par, prec="f16").cpu().numpy()
        mats, nbr = lowprec.site_matrices(fat, lng, dims, par, cbs=sample)
        sc = lowprec.folded_scalars(dims, par, cbs=sample) if long12 else None
        mats_q = lowprec.round_matrices(mats, "f16", long12=long12, scalars=sc)
        uniq, inv = np.unique(nbr, return_inverse=True)
        inv = inv.reshape(nbr.shape)
        for r in range(b.shape[0]):
            b_q = lowprec.round_spinor(b[r][uniq], "f16")
            ref = lowprec.apply_site_matrices(mats_q, inv, b_q)
            s = np.max(np.abs(np.stack([ref.real, ref.imag], -1)).reshape(len(ref), -1), axis=1)
            bound = c * u32 * lowprec.abs_bound_terms(mats_q, inv, b_q) + (2.0 ** -11) * s[:, None] * 1.001
            got = out[r][sample]
            assert np.all(np.abs(got.real - ref.real) <= bound), (par, r)
            assert np.all(np.abs(got.imag - ref.imag) <= bound), (par, r)
            # the result is the rounded operator's, not the exact one
            assert rel(got, dslash_at_sites(fat, lng, b[r], dims, par, sample)) > 1e-8
        outs.append(out)
    return outs


def test_large_lattice_f16_dslash_sampled_in_benchmark_shapes(gpu_lib, c5):
    """48^3x144 x 8 RHS, FP16 storage: the kernel the benchmark times (18-real three-hop links, 128-site
    workgroups, 8 RHS per lane, XCD z-block order) and the 12-real form in its default shape, against the
    low-precision oracle at sampled sites (tile edges and wraps included); every other launch shape of
    the same storage gives bitwise the same result."""
    lat, fat, lng, b, bt, dims, nrhs = (c5[k] for k in ("lat", "fat", "lng", "b", "bt", "dims", "nrhs"))
    half = b.shape[1]
    rng = np.random.default_rng(6)
    sample = np.concatenate([rng.integers(0, half, 96), np.arange(32), np.arange(half - 32, half),
                             half // 2 + np.arange(-8, 8)])
    for long12, shapes in ((False, ((128, 8, 0, 1, 1), (64, 8, 0, 1, 3), (64, 4, 0, 0), (64, 8, 0, 2, 2))),
                           (True, ((64, 4, 0, 1), (64, 1, 0, 0), (64, 8, 0, 2, 1)))):
        print(f"48^3x144 sampled f16 dslash, {'12' if long12 else '18'}-real three-hop links", flush=True)
        lat.load_links(torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda(), NAIK, precs=("f64", "f16"),
                       long_su3=long12)
        torch.cuda.empty_cache()
        lat.set_dslash_shape("f16", nrhs, *shapes[0])
        outs = _f16_sampled_check(lat, fat, lng, b, bt, dims, sample, long12)
        for shape in shapes[1:]:
            lat.set_dslash_shape("f16", nrhs, *shape)
            for par in (0, 1):
                assert np.array_equal(lat.dslash(bt, par, prec="f16").cpu().numpy(), outs[par]), shape
        lat.set_dslash_shape("f16", nrhs, 0, 1)
