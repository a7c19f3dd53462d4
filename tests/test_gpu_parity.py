"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded inputs."""
import numpy as np
import pytest
import torch

from oracle import lowprec
from oracle.cg import cg, true_residual
from oracle.dslash import apply_m, dslash_at_sites, dslash_eo
from stag_inputs import fat_field, gaussian_source, random_su3_field

pytestmark = pytest.mark.gpu

NAIK = -1.0 / 24.0


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make(dims, seed=5, naik=True, precs=("f64",), antiperiodic=True):
    from paper_1010_4782_amd.stagcg import Lattice

    fat = fat_field(dims, seed)
    lng = random_su3_field(dims, seed + 1) if naik else None
    lat = Lattice(dims, antiperiodic)
    lat.load_links(torch.from_numpy(fat).cuda(), None if lng is None else torch.from_numpy(lng).cuda(),
                   NAIK, precs=precs)
    return lat, fat, lng


DIMS = [(2, 2, 2, 2), (4, 4, 4, 4), (2, 4, 6, 8), (6, 6, 6, 6), (8, 8, 8, 8), (10, 4, 2, 6), (4, 2, 8, 2)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("nrhs", [1, 3, 4])
def test_dslash_f64_matches_oracle(gpu_lib, dims, nrhs):
    print(f"dslash f64 dims={dims} nrhs={nrhs}", flush=True)
    lat, fat, lng = make(dims)
    b = gaussian_source(dims, 11, nrhs)
    x = torch.from_numpy(b).cuda()
    for par in (0, 1):
        out = lat.dslash(x, par).cpu().numpy()
        for r in range(nrhs):
            ref = dslash_eo(fat, lng, b[r], dims, par)
            assert rel(out[r], ref) <= 1e-12, (par, r)


@pytest.mark.parametrize("nrhs", [2, 8])
def test_dslash_f64_multi_rhs_groups(gpu_lib, nrhs):
    dims = (6, 4, 4, 6)
    print(f"dslash f64 multi-rhs dims={dims} nrhs={nrhs}", flush=True)
    lat, fat, lng = make(dims, seed=21)
    b = gaussian_source(dims, 12, nrhs)
    out = lat.dslash(torch.from_numpy(b).cuda(), 1).cpu().numpy()
    for r in range(nrhs):
        assert rel(out[r], dslash_eo(fat, lng, b[r], dims, 1)) <= 1e-12


@pytest.mark.parametrize("antiperiodic", [True, False])
def test_dslash_one_hop_and_periodic(gpu_lib, antiperiodic):
    """No long links (the paper's Eq. (5) alone), both time boundary conditions."""
    dims = (4, 6, 4, 8)
    print(f"dslash one-hop antiperiodic={antiperiodic}", flush=True)
    lat, fat, _ = make(dims, naik=False, antiperiodic=antiperiodic)
    b = gaussian_source(dims, 13)[0]
    out = lat.dslash(torch.from_numpy(b).cuda(), 0).cpu().numpy()
    ref = dslash_eo(fat, None, b, dims, 0, antiperiodic_t=antiperiodic)
    assert rel(out, ref) <= 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 6, 6, 6), (2, 4, 6, 8)])
def test_apply_m_matches_oracle(gpu_lib, dims):
    print(f"apply_m dims={dims}", flush=True)
    lat, fat, lng = make(dims)
    b = gaussian_source(dims, 14, 2)
    masses = [0.05, 0.3]
    out = lat.apply_m(torch.from_numpy(b).cuda(), masses).cpu().numpy()
    for r in range(2):
        assert rel(out[r], apply_m(fat, lng, b[r], dims, masses[r])) <= 1e-12


@pytest.mark.parametrize("prec", ["f32", "f16"])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 6, 6, 6), (2, 4, 6, 8)])
def test_dslash_lowprec_within_bound(gpu_lib, prec, dims):
    """Low-precision Dslash vs the oracle on identically rounded inputs, within a derived rounding bound.

    FP32 arithmetic over 16 links x 3 colours (48 complex products, 4 FMAs each) is
    bounded by gamma_200 ~ 200 u_32 sum |terms| per component; an FP16 output adds
    half a binary16 spacing of the site scale, at most 2^-11 s.
    """
    print(f"dslash {prec} dims={dims}", flush=True)
    lat, fat, lng = make(dims, precs=("f64", prec))
    b = gaussian_source(dims, 15)[0]
    u32 = 2.0 ** -24
    for par in (0, 1):
        out = lat.dslash(torch.from_numpy(b).cuda(), par, prec=prec).cpu().numpy()
        mats, nbr = lowprec.site_matrices(fat, lng, dims, par)
        mats_q = lowprec.round_matrices(mats, prec)
        b_q = lowprec.round_spinor(b, prec)
        ref = lowprec.apply_site_matrices(mats_q, nbr, b_q)
        A = lowprec.abs_bound_terms(mats_q, nbr, b_q)
        bound = 200 * u32 * A
        if prec == "f16":
            s = np.max(np.abs(np.stack([ref.real, ref.imag], -1)).reshape(len(ref), -1), axis=1)
            bound = bound + (2.0 ** -11) * s[:, None] * 1.001
        assert np.all(np.abs(out.real - ref.real) <= bound), (par, float((np.abs(out.real - ref.real) / bound).max()))
        assert np.all(np.abs(out.imag - ref.imag) <= bound), par
        # and the rounding actually happened: the result differs from the exact FP64 operator
        assert rel(out, dslash_eo(fat, lng, b, dims, par)) > 1e-10


def test_cg_f64_matches_oracle_iterates(gpu_lib):
    """8^4, m = 0.05 (the small-lattice workload): GPU FP64 CG vs the oracle's Fig. 1 loop."""
    dims = (8, 8, 8, 8)
    print("cg f64 8^4", flush=True)
    from paper_1010_4782_amd.stagcg import Lattice

    fat = random_su3_field(dims, 1001)  # unitary one-hop links for this workload
    lng = random_su3_field(dims, 1002)
    lat = Lattice(dims)
    lat.load_links(torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda(), NAIK)
    m = 0.05
    b = gaussian_source(dims, 1010)[0]
    A = lambda v: apply_m(fat, lng, v, dims, m)
    ref = cg(A, b, tol=1e-10, record=10)
    hist = np.zeros((1, 10, 2))
    x, info = lat.cg_solve(torch.from_numpy(b).cuda(), m, tol=1e-10, history_len=10, history=hist)
    x = x.cpu().numpy()
    assert info[0]["converged"] == 1
    assert info[0]["true_resid"] <= 1e-10
    assert true_residual(A, b, x) <= 1.05e-10
    assert abs(info[0]["iters"] - ref.iters) <= max(5, 0.02 * ref.iters)
    np.testing.assert_allclose(hist[0, :, 0], ref.alphas, rtol=1e-10)
    np.testing.assert_allclose(hist[0, :, 1], ref.betas, rtol=1e-10)


def test_cg_first_step_scalars_many_partials(gpu_lib):
    """36^3 x 72 with 64-site operator workgroups: <d, Ad> arrives as 26,244 partials, more than the
    24,576 one pass of the device-side finalize sums, so the second (ragged) pass is exercised.
    alpha_0 = |b|^2 / <b, M b> and beta_0 = |b - alpha_0 M b|^2 / |b|^2 (Fig. 1 with x0 = 0) from
    the oracle's own M.  The links are complex Gaussian matrices (any links keep D_eo = -D_oe^dagger,
    so M stays Hermitian positive definite), cheaper to draw at this size than SU(3) fields."""
    from paper_1010_4782_amd.stagcg import Lattice

    dims = (36, 36, 36, 72)
    print(f"cg first-step scalars {dims}", flush=True)
    rng = np.random.default_rng(3601)
    shp = (4, dims[3], dims[2], dims[1], dims[0], 3, 3)
    fat = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * 0.4
    lng = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * 0.4
    b = gaussian_source(dims, 3610)[0]
    m = 0.0062
    lat = Lattice(dims)
    lat.load_links(torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda(), NAIK)
    lat.set_dslash_shape("f64", 1, 64, 1)
    assert -(-len(b) // 64) > 24576
    hist = np.zeros((1, 2, 2))
    _, info = lat.cg_solve(torch.from_numpy(b).cuda(), m, max_iter=2, max_restarts=0, history_len=2,
                           history=hist, raise_on_fail=False)
    assert info[0]["iters"] == 2
    Mb = apply_m(fat, lng, b, dims, m)
    b2 = np.vdot(b, b).real
    alpha0 = b2 / np.vdot(b, Mb).real
    r1 = b - alpha0 * Mb
    beta0 = np.vdot(r1, r1).real / b2
    np.testing.assert_allclose(hist[0, 0], [alpha0, beta0], rtol=1e-11)
    lat.set_dslash_shape("f64", 1, 0, 1)


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_cg_mixed_precision_true_residual(gpu_lib, prec):
    dims = (8, 8, 8, 8)
    print(f"cg {prec} 8^4", flush=True)
    lat, fat, lng = make(dims, seed=31, precs=("f64", prec))
    m = 0.05
    b = gaussian_source(dims, 32, 2)
    x, info = lat.cg_solve(torch.from_numpy(b).cuda(), [m, 0.1], tol=1e-10, prec=prec, reliable_interval=50)
    x = x.cpu().numpy()
    for r, mr in enumerate([m, 0.1]):
        assert info[r]["converged"] == 1 and info[r]["n_reliable"] >= 1
        assert true_residual(lambda v: apply_m(fat, lng, v, dims, mr), b[r], x[r]) <= 1.05e-10


def test_reliable_update_interval_is_exact(gpu_lib):
    """With the residual-drop trigger off, the FP64 reliable update comes every reliable_interval inner
    iterations, even when that is not a multiple of the polling interval (20 vs 16 here)."""
    dims = (8, 8, 8, 8)
    print("reliable interval 8^4", flush=True)
    lat, fat, lng = make(dims, seed=33, precs=("f64", "f16"))
    b = gaussian_source(dims, 34, 1)
    m = 0.05
    x, info = lat.cg_solve(torch.from_numpy(b).cuda(), m, tol=1e-10, prec="f16", reliable_interval=20,
                           reliable_delta=0.0, check_interval=16)
    it, nrel = info[0]["iters"], info[0]["n_reliable"]
    assert info[0]["converged"] == 1 and it >= 40, info[0]
    # one update per 20 iterations, plus at most one at apparent convergence (a multiple of 16 would give
    # one per 32)
    assert it // 20 <= nrel <= it // 20 + 2, (it, nrel)
    assert true_residual(lambda v: apply_m(fat, lng, v, dims, m), b[0], x.cpu().numpy()[0]) <= 1.05e-10


def test_cg_batched_uneven_lattices(gpu_lib):
    from paper_1010_4782_amd.stagcg import cg_solve_batch

    print("cg batch uneven", flush=True)
    probs, refs = [], []
    for i, (dims, nrhs) in enumerate([((4, 4, 4, 4), 2), ((6, 4, 4, 6), 4), ((8, 8, 8, 8), 1)]):
        lat, fat, lng = make(dims, seed=40 + i, precs=("f64", "f32"))
        b = gaussian_source(dims, 50 + i, nrhs)
        masses = [0.05 + 0.05 * r for r in range(nrhs)]
        probs.append((lat, torch.from_numpy(b).cuda(), masses, None))
        refs.append((fat, lng, dims, b, masses))
    for prec in ("f64", "f32"):
        xs, infos = cg_solve_batch(probs, tol=1e-10, prec=prec)
        k = 0
        for (fat, lng, dims, b, masses), x in zip(refs, xs):
            x = x.cpu().numpy()
            for r, mr in enumerate(masses):
                assert infos[k]["converged"] == 1
                assert true_residual(lambda v: apply_m(fat, lng, v, dims, mr), b[r], x[r]) <= 1.05e-10
                k += 1


def test_cg_edge_cases(gpu_lib):
    from paper_1010_4782_amd._lib import STAG_ERR_NOT_CONVERGED, StagError

    print("cg edge cases", flush=True)
    dims = (4, 4, 4, 4)
    lat, fat, lng = make(dims, seed=61)
    b = gaussian_source(dims, 62, 2)
    b[1] = 0.0                                   # zero source -> x = 0 exactly
    bt = torch.from_numpy(b).cuda()
    x, info = lat.cg_solve(bt, 0.1)
    assert info[1]["iters"] == 0 and not x[1].abs().max().item()
    # warm start at the solution: no iterations
    x2, info2 = lat.cg_solve(bt[:1].contiguous(), 0.1, x0=x[:1].contiguous())
    assert info2[0]["iters"] == 0 and info2[0]["converged"] == 1
    # iteration cap reached: STAG_ERR_NOT_CONVERGED with a finite last iterate
    x3, info3 = lat.cg_solve(bt[:1].contiguous(), 0.01, max_iter=3, max_restarts=0, raise_on_fail=False)
    assert info3[0]["status"] == STAG_ERR_NOT_CONVERGED and info3[0]["iters"] == 3
    assert torch.isfinite(x3).all()
    with pytest.raises(StagError):
        lat.cg_solve(bt[:1].contiguous(), 0.01, max_iter=3, max_restarts=0)


def test_cg_degenerate_cases(gpu_lib):
    """Massless operator (M = D_oe^dag D_oe, positive semi-definite), a non-finite source, and a zero
    source in mixed precision."""
    from paper_1010_4782_amd._lib import STAG_ERR_NAN

    print("cg degenerate cases", flush=True)
    dims = (4, 4, 4, 4)
    lat, fat, lng = make(dims, seed=71, precs=("f64", "f16"))
    b = gaussian_source(dims, 72, 1)
    x, info = lat.cg_solve(torch.from_numpy(b).cuda(), 0.0, tol=1e-10)
    assert info[0]["converged"] == 1
    assert true_residual(lambda v: apply_m(fat, lng, v, dims, 0.0), b[0], x[0].cpu().numpy()) <= 1.05e-10
    bn = b.copy()
    bn[0, 5, 1] = np.nan
    xn, infon = lat.cg_solve(torch.from_numpy(bn).cuda(), 0.1, raise_on_fail=False)
    assert infon[0]["status"] == STAG_ERR_NAN and infon[0]["converged"] == 0
    z = torch.zeros_like(torch.from_numpy(b)).cuda()
    xz, infoz = lat.cg_solve(z, 0.1, prec="f16")
    assert infoz[0]["iters"] == 0 and not xz.abs().max().item()


def test_solves_are_deterministic(gpu_lib):
    dims = (6, 6, 6, 6)
    print("determinism", flush=True)
    lat, _, _ = make(dims, seed=71)
    bt = torch.from_numpy(gaussian_source(dims, 72)).cuda()
    x1, i1 = lat.cg_solve(bt, 0.05)
    x2, i2 = lat.cg_solve(bt, 0.05)
    assert torch.equal(x1, x2) and i1[0]["iters"] == i2[0]["iters"]


def test_argument_errors(gpu_lib):
    from paper_1010_4782_amd._lib import StagError
    from paper_1010_4782_amd.stagcg import Lattice

    with pytest.raises(StagError):
        Lattice((3, 4, 4, 4))
    lat = Lattice((4, 4, 4, 4))
    v = torch.zeros(128, 3, dtype=torch.complex128, device="cuda")
    with pytest.raises(StagError):
        lat.dslash(v, 0)                        # links not loaded yet
    lat2, _, _ = make((4, 4, 4, 4))
    with pytest.raises(StagError):
        lat2.dslash(v, 0, prec="f16")           # precision not packed
    # b and x overlapping (the binding never does this; the C ABI must refuse it)
    import ctypes as C

    from paper_1010_4782_amd._lib import StagInfo, lib
    from paper_1010_4782_amd.stagcg import solve_params

    prm = solve_params()
    info = (StagInfo * 1)()
    mass = (C.c_double * 1)(0.1)
    st = lib().stag_cg_solve(lat2.handle, mass, C.c_void_p(v.data_ptr()), C.c_void_p(v.data_ptr()), 1,
                             C.byref(prm), info, None)
    assert st == 1  # STAG_ERR_ARG


@pytest.mark.parametrize("long_su3", [False, True])
def test_dslash_full_size_28cubed_96_sampled(gpu_lib, long_su3):
    """The paper-shaped lattice 28^3 x 96 in the launch shape the solver uses: sampled sites vs the oracle."""
    dims = (28, 28, 28, 96)
    print(f"dslash 28^3x96 sampled long_su3={long_su3}", flush=True)
    fat = fat_field(dims, 2001)
    lng = random_su3_field(dims, 2002)
    from paper_1010_4782_amd.stagcg import Lattice

    lat = Lattice(dims)
    lat.load_links(torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda(), NAIK, precs=("f64", "f16"),
                   long_su3=long_su3)
    b = gaussian_source(dims, 2010)[0]
    rng = np.random.default_rng(3)
    half = len(b)
    sample = np.concatenate([rng.integers(0, half, 400), np.arange(64), np.arange(half - 64, half)])
    for par in (0, 1):
        out = lat.dslash(torch.from_numpy(b).cuda(), par).cpu().numpy()
        ref = dslash_at_sites(fat, lng, b, dims, par, sample)
        assert rel(out[sample], ref) <= 1e-12


def test_dslash_identical_for_every_launch_shape(gpu_lib):
    """Workgroup size, right-hand sides per lane and LDS staging change the schedule, not the arithmetic:
    bitwise equal."""
    from paper_1010_4782_amd._lib import StagError

    dims = (6, 4, 6, 8)
    print("dslash launch shapes", flush=True)
    lat, fat, lng = make(dims, seed=91, precs=("f64", "f32", "f16"))
    b = torch.from_numpy(gaussian_source(dims, 92, 8)).cuda()
    for prec in ("f64", "f32", "f16"):
        ref = None
        for wg in (64, 128, 256):
            for r in (1, 2, 4, 8):
                for lds in (0, 1):
                    if lds and r * (wg + 3 * dims[0]) * {"f64": 48, "f32": 24, "f16": 16}[prec] > 65536:
                        with pytest.raises(StagError):  # the staged window would not fit in 64 KiB of LDS
                            lat.set_dslash_shape(prec, 8, wg, r, lds)
                        continue
                    lat.set_dslash_shape(prec, 8, wg, r, lds)
                    out = lat.dslash(b, 1, prec=prec)
                    if ref is None:
                        ref = out.clone()
                    assert torch.equal(out, ref), (prec, wg, r, lds)
        lat.set_dslash_shape(prec, 8, 0, 1)
    assert rel(ref.cpu().numpy()[3], dslash_eo(fat, lng, b.cpu().numpy()[3], dims, 1)) > 0  # f16 result exists
    best, timed = lat.tune_dslash("f16", 8)
    assert best[0] in (64, 128, 256) and best[1] in (1, 2, 4, 8) and best[2] in (0, 1) and len(timed) == 24
    # neither the XCD-block order (Lz = 6) nor the time-streaming kernel (72 sites per slice) fits
    assert best[3] == 0 and all(t[3] == 0 and t[5] > 0 for t in timed)


def test_xcd_block_tile_order_is_bitwise_equal(gpu_lib):
    """The XCD-block tile order only changes which workgroup takes which tile: every shape gives the bits
    of the lattice order, and a lattice or workgroup size it does not fit is refused."""
    from paper_1010_4782_amd._lib import StagError

    dims = (8, 16, 8, 4)  # Lz = 8 blocks of one z plane; Ly x Lx / 2 = 64 sites per z plane
    print("dslash tile order", flush=True)
    lat, fat, lng = make(dims, seed=93, precs=("f64", "f16"))
    b = torch.from_numpy(gaussian_source(dims, 94, 4)).cuda()
    for prec in ("f64", "f16"):
        lat.set_dslash_shape(prec, 4, 64, 1)
        ref = lat.dslash(b, 0, prec=prec)
        for r in (1, 2, 4):
            for lds in (0, 1):
                lat.set_dslash_shape(prec, 4, 64, r, lds, 1)
                assert torch.equal(lat.dslash(b, 0, prec=prec), ref), (prec, r, lds)
        with pytest.raises(StagError):
            lat.set_dslash_shape(prec, 4, 128, 1, 0, 1)  # 128 does not divide the 64 sites of a z plane
        with pytest.raises(StagError):
            lat.set_dslash_shape(prec, 4, 64, 1, 0, 1, 2)  # Lz = 8 cannot be cut into 16 blocks
        lat.set_dslash_shape(prec, 4, 0, 1)
    assert rel(ref.cpu().numpy()[1], dslash_eo(fat, lng, b.cpu().numpy()[1], dims, 0)) > 0
    x, info = lat.cg_solve(b, 0.05, tol=1e-10, prec="f16")
    assert all(i["converged"] == 1 for i in info)
    # thinner blocks: Lz = 48 in 8, 16, 24 or 48 blocks (one z plane per block)
    dims = (8, 16, 48, 2)
    lat, _, _ = make(dims, seed=95, precs=("f64", "f16"))
    b = torch.from_numpy(gaussian_source(dims, 96, 8)).cuda()
    for prec in ("f64", "f16"):
        lat.set_dslash_shape(prec, 8, 64, 1)
        ref = lat.dslash(b, 1, prec=prec)
        for c in (1, 2, 3, 6):
            for r in (1, 4, 8):
                lat.set_dslash_shape(prec, 8, 64, r, 0, 1, c)
                assert torch.equal(lat.dslash(b, 1, prec=prec), ref), (prec, r, c)
        with pytest.raises(StagError):
            lat.set_dslash_shape(prec, 8, 64, 1, 0, 1, 4)  # 48 is not a multiple of 32 blocks
        lat.set_dslash_shape(prec, 8, 0, 1)


def test_batched_solve_with_autotune(gpu_lib):
    from paper_1010_4782_amd.stagcg import cg_solve_batch

    print("batched solve autotune", flush=True)
    probs, refs = [], []
    for i, (dims, nrhs) in enumerate([((4, 4, 4, 8), 4), ((6, 6, 4, 4), 8)]):
        lat, fat, lng = make(dims, seed=95 + i, precs=("f64", "f16"))
        b = gaussian_source(dims, 97 + i, nrhs)
        probs.append((lat, torch.from_numpy(b).cuda(), [0.05] * nrhs, None))
        refs.append((fat, lng, dims, b))
    xs, infos = cg_solve_batch(probs, tol=1e-10, prec="f16", autotune=True)
    assert infos[0]["dslash_rhs"] in (1, 2, 4, 8)
    k = 0
    for (fat, lng, dims, b), x in zip(refs, xs):
        x = x.cpu().numpy()
        for r in range(len(b)):
            assert infos[k]["converged"] == 1
            assert true_residual(lambda v: apply_m(fat, lng, v, dims, 0.05), b[r], x[r]) <= 1.05e-10
            k += 1


def make12(dims, seed, precs):
    from paper_1010_4782_amd.stagcg import Lattice

    fat = fat_field(dims, seed)
    lng = random_su3_field(dims, seed + 1)
    lat = Lattice(dims)
    lat.load_links(torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda(), NAIK, precs=precs, long_su3=True)
    return lat, fat, lng


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 6, 6, 6), (2, 4, 6, 8), (4, 2, 8, 2)])
def test_dslash_f64_twelve_parameter_long_links(gpu_lib, dims):
    """Long links stored as two rows (Sec. 3.3): FP64 Dslash still matches the exact operator to 1e-12."""
    print(f"dslash f64 long12 {dims}", flush=True)
    lat, fat, lng = make12(dims, 101, ("f64",))
    b = gaussian_source(dims, 102, 2)
    for par in (0, 1):
        out = lat.dslash(torch.from_numpy(b).cuda(), par).cpu().numpy()
        for r in range(2):
            assert rel(out[r], dslash_eo(fat, lng, b[r], dims, par)) <= 1e-12


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_dslash_lowprec_twelve_parameter_within_bound(gpu_lib, prec):
    dims = (6, 4, 4, 6)
    print(f"dslash {prec} long12", flush=True)
    lat, fat, lng = make12(dims, 103, ("f64", prec))
    b = gaussian_source(dims, 104)[0]
    u32 = 2.0 ** -24
    for par in (0, 1):
        out = lat.dslash(torch.from_numpy(b).cuda(), par, prec=prec).cpu().numpy()
        mats, nbr = lowprec.site_matrices(fat, lng, dims, par)
        sc = lowprec.folded_scalars(dims, par)
        mats_q = lowprec.round_matrices(mats, prec, long12=True, scalars=sc)
        b_q = lowprec.round_spinor(b, prec)
        ref = lowprec.apply_site_matrices(mats_q, nbr, b_q)
        # rebuilding the third row in binary32 adds a few more roundings per three-hop term
        bound = 300 * u32 * lowprec.abs_bound_terms(mats_q, nbr, b_q)
        if prec == "f16":
            s = np.max(np.abs(np.stack([ref.real, ref.imag], -1)).reshape(len(ref), -1), axis=1)
            bound = bound + (2.0 ** -11) * s[:, None] * 1.001
        assert np.all(np.abs(out.real - ref.real) <= bound), (par, float((np.abs(out.real - ref.real) / bound).max()))
        assert np.all(np.abs(out.imag - ref.imag) <= bound), par


@pytest.mark.parametrize("prec", ["f64", "f16"])
def test_cg_with_twelve_parameter_long_links(gpu_lib, prec):
    dims = (8, 8, 8, 8)
    print(f"cg long12 {prec}", flush=True)
    lat, fat, lng = make12(dims, 105, ("f64", "f16"))
    m = 0.05
    b = gaussian_source(dims, 106)
    x, info = lat.cg_solve(torch.from_numpy(b).cuda(), m, prec=prec)
    assert info[0]["converged"] == 1
    assert true_residual(lambda v: apply_m(fat, lng, v, dims, m), b[0], x.cpu().numpy()[0]) <= 1.05e-10


def test_profile_samples_every_kth_iteration(gpu_lib):
    """profile = k brackets the Dslash pair of every k-th iteration: 2 launches per sampled iteration."""
    lat, fat, lng = make((6, 6, 6, 6), seed=111, precs=("f64",))
    b = torch.from_numpy(gaussian_source((6, 6, 6, 6), 112)).cuda()
    print("profile sampling", flush=True)
    _, info1 = lat.cg_solve(b, 0.1, tol=1e-10, profile=1)
    _, info5 = lat.cg_solve(b, 0.1, tol=1e-10, profile=5)
    _, info0 = lat.cg_solve(b, 0.1, tol=1e-10, profile=0)
    it = info1[0]["iters"]
    assert info1[0]["iters"] == info5[0]["iters"] == info0[0]["iters"]  # timing does not change the solve
    # iterations are launched in chunks of 16 between polls, so up to 15 launched after convergence
    # may be sampled too (on a lattice this small they are not told apart from working ones)
    for k, info in ((1, info1), (5, info5)):
        lo, hi = 2 * (-(-it // k)) - 4, 2 * (-(-(it + 15) // k)) + 4
        assert lo <= info[0]["dslash_calls"] <= hi, (k, it, info[0]["dslash_calls"])
    assert info0[0]["dslash_calls"] == 0 and info0[0]["dslash_ms"] == 0.0
    assert info1[0]["dslash_ms"] > 0 and info5[0]["dslash_ms"] > 0


def test_batch_rejects_mixed_long_link_storage(gpu_lib):
    """One launch per stage serves every lattice of a batch, so their three-hop storage must agree."""
    from paper_1010_4782_amd.stagcg import StagError, cg_solve_batch

    print("mixed long-link batch", flush=True)
    dims = (4, 4, 4, 4)
    lat_a, _, _ = make(dims, seed=121, precs=("f64",))
    lat_b, _, _ = make12(dims, 123, ("f64",))
    b = torch.from_numpy(gaussian_source(dims, 125)).cuda()
    with pytest.raises(StagError):
        cg_solve_batch([(lat_a, b, [0.1], None), (lat_b, b, [0.1], None)], tol=1e-10)


@pytest.mark.parametrize("prec,long_su3", [("f64", False), ("f64", True), ("f16", True)])
def test_dslash_slab_loopback_equals_unsplit(gpu_lib, prec, long_su3):
    """Domain decomposition along t on one GPU: each slab of lt slices gets its two 3-slice faces from
    its neighbours (a contiguous copy each; the antiperiodic wrap included) and applies the Dslash;
    the assembled slabs equal the unsplit operator bit for bit."""
    dims = (6, 4, 4, 16)
    print(f"dslash slab loopback {prec} long_su3={long_su3}", flush=True)
    lat, fat, lng = (make12(dims, 131, ("f64", "f16")) if long_su3 else make(dims, seed=131, precs=("f64", "f16")))
    S = dims[0] * dims[1] * dims[2] // 2
    Lt = dims[3]
    b = torch.from_numpy(gaussian_source(dims, 133, 2)).cuda()
    refs = {}
    # the default shape, then both RHS on one lane with the x/y neighbour window staged in LDS (the slab's
    # input has 6 more slices than its output: the window is indexed in the input's sites)
    for shape in (None, (256, 2, 1)):
        if shape:
            lat.set_dslash_shape(prec, 2, *shape)
        for par in (0, 1):
            ref = lat.dslash(b, par, prec=prec)
            assert torch.equal(refs.setdefault(par, ref), ref), (par, shape)
            for lt in (4, 8):
                for t0 in range(0, Lt, lt):
                    # the slab's extended input: slices t0-3 .. t0+lt+2 (mod Lt), faces copied from the neighbours
                    rows = torch.cat([torch.arange(((t0 + k) % Lt) * S, ((t0 + k) % Lt + 1) * S)
                                      for k in range(-3, lt + 3)])
                    ext = b[:, rows.cuda(), :].contiguous()
                    out = lat.dslash_slab(ext, par, t0, lt, prec=prec)
                    assert torch.equal(out, ref[:, t0 * S:(t0 + lt) * S, :]), (par, lt, t0, shape)
    lat.set_dslash_shape(prec, 2, 0, 1)
    from paper_1010_4782_amd.stagcg import StagError

    with pytest.raises(StagError):  # odd t0: the slab would change the even-odd parity of its sites
        lat.dslash_slab(torch.zeros((1, 10 * S, 3), dtype=torch.complex128, device="cuda"), 0, 1, 4)


def test_pion_correlator_of_point_source_propagators(gpu_lib):
    """Point sources at two even sites (three colours each) solved on the GPU; the correlator from
    stag_slice_norm2 and the GPU Dslash against the oracle, on the GPU's own solution (the sums) and on
    the oracle's solution (the whole chain), plus the sum rule sum_t C(t) = sum_c chi^(c)(x0)_c."""
    from oracle import geometry
    from oracle.propagator import correlator, even_solutions, propagator
    from stag_inputs import point_sources

    dims = (4, 4, 4, 8)
    m = 0.1
    print("pion correlator 4^3x8", flush=True)
    lat, fat, lng = make(dims, seed=321, precs=("f64", "f16"))
    sites = [(0, 0, 0, 0), (1, 2, 3, 2)]
    b = point_sources(dims, sites)
    bt = torch.from_numpy(b).cuda()
    chi, info = lat.cg_solve(bt, m, tol=1e-12)
    assert all(i["converged"] == 1 for i in info)
    C = lat.pion_correlator(chi, m).cpu().numpy()
    chi_h = chi.cpu().numpy()
    np.testing.assert_allclose(C, correlator(*propagator(fat, lng, dims, m, chi_h), dims), rtol=1e-12)
    ref = correlator(*propagator(fat, lng, dims, m, even_solutions(fat, lng, dims, m, b, tol=1e-13)), dims)
    np.testing.assert_allclose(C, ref, rtol=1e-9)
    for s, site in enumerate(sites):
        cb = geometry.cb_of_site(*site, dims)
        assert C[s].sum() == pytest.approx(sum(chi_h[3 * s + c, cb, c].real for c in range(3)), rel=1e-10)
    # the mixed-precision solve gives the same correlator to the accuracy of its solution
    chi16, info16 = lat.cg_solve(bt, m, tol=1e-10, prec="f16")
    np.testing.assert_allclose(lat.pion_correlator(chi16, m).cpu().numpy(), ref, rtol=1e-7)
    # the sums honour group and accumulate; a group that does not divide nrhs is refused
    one = lat.slice_norm2(chi, 1, 2.0).cpu().numpy()
    np.testing.assert_allclose(one[0] + one[1] + one[2], lat.slice_norm2(chi, 3, 2.0).cpu().numpy()[0], rtol=1e-13)
    from paper_1010_4782_amd._lib import StagError

    with pytest.raises((StagError, ValueError)):
        lat.slice_norm2(chi, 4)


@pytest.mark.parametrize("dims,long_su3", [((8, 4, 4, 6), True), ((4, 4, 4, 8), True), ((4, 4, 4, 2), True),
                                           ((8, 8, 4, 4), False), ((16, 4, 4, 4), True)])
def test_time_streaming_dslash_is_bitwise_equal(gpu_lib, dims, long_su3):
    """The time-streaming FP16 kernel (8 or 4 RHS per lane, the time extent in 1..Lt/2 chunks) against the
    site-parallel kernel: the same matrices in the same order, so the same bits, for 8 and 16 RHS and both
    output parities; on Lt = 2, 4, 6 the time hops wrap one to three times.  Shapes whose site count per
    slice is not a multiple of the wave's sites are refused."""
    from paper_1010_4782_amd._lib import StagError

    print(f"time-streaming dslash {dims} long_su3={long_su3}", flush=True)
    lat, fat, lng = make12(dims, 141, ("f64", "f16")) if long_su3 else make(dims, seed=141, precs=("f64", "f16"))
    S = dims[0] * dims[1] * dims[2] // 2
    b = torch.from_numpy(gaussian_source(dims, 142, 16)).cuda()
    for nrhs in (8, 16):
        bn = b[:nrhs].contiguous()
        for par in (0, 1):
            lat.set_dslash_shape("f16", nrhs, 64, 8)
            ref = lat.dslash(bn, par, prec="f16")
            for r in (8, 4):
                for chunks in range(1, dims[3] // 2 + 1):
                    if (dims[3] // 2) % chunks:
                        continue
                    if S % (64 * r // 8):
                        with pytest.raises(StagError):
                            lat.set_dslash_shape("f16", nrhs, 64, r, 0, 2, chunks)
                        continue
                    lat.set_dslash_shape("f16", nrhs, 64, r, 0, 2, chunks)
                    assert torch.equal(lat.dslash(bn, par, prec="f16"), ref), (nrhs, par, r, chunks)
        lat.set_dslash_shape("f16", nrhs, 0, 1)
    with pytest.raises(StagError):  # 12 RHS: not a multiple of 8
        lat.set_dslash_shape("f16", 12, 64, 8, 0, 2, 1)
    with pytest.raises(StagError):  # FP64 has no time-streaming kernel
        lat.set_dslash_shape("f64", 8, 64, 8, 0, 2, 1)


def test_time_streaming_solve(gpu_lib):
    """Mixed-precision CG with the time-streaming kernel in its iterations: with 8 RHS per lane its
    reduction partials are those of a 64-site workgroup, so the solve gives the bits of the site-parallel
    kernel's; with 4 RHS per lane (32-site partials) it converges to the same true residual (oracle).
    Per-RHS masses make the right-hand sides stop at different iterations, which exercises the
    per-lane convergence masks; two lattices in one batch exercise the problem table."""
    from paper_1010_4782_amd.stagcg import cg_solve_batch

    dims = (8, 8, 4, 8)
    print("time-streaming solve", flush=True)
    lat, fat, lng = make12(dims, 151, ("f64", "f16"))
    b = gaussian_source(dims, 152, 8)
    bt = torch.from_numpy(b).cuda()
    masses = [0.05, 0.08, 0.1, 0.2, 0.3, 0.05, 0.12, 0.5]
    lat.set_dslash_shape("f16", 8, 64, 8)
    x0, i0 = lat.cg_solve(bt, masses, tol=1e-10, prec="f16")
    lat.set_dslash_shape("f16", 8, 64, 8, 0, 2, 2)
    x1, i1 = lat.cg_solve(bt, masses, tol=1e-10, prec="f16")
    assert torch.equal(x0, x1) and [i["iters"] for i in i0] == [i["iters"] for i in i1]
    assert len(set(i["iters"] for i in i1)) > 2  # the RHS stopped at different iterations
    lat.set_dslash_shape("f16", 8, 64, 4, 0, 2, 1)
    x2, i2 = lat.cg_solve(bt, masses, tol=1e-10, prec="f16")
    x2 = x2.cpu().numpy()
    for r, m in enumerate(masses):
        assert i2[r]["converged"] == 1
        assert true_residual(lambda v: apply_m(fat, lng, v, dims, m), b[r], x2[r]) <= 1.05e-10
    lat.set_dslash_shape("f16", 8, 0, 1)
    # two lattices in one batch, both in the time-streaming kernel
    dims2 = (8, 4, 4, 6)
    lat2, fat2, lng2 = make12(dims2, 153, ("f64", "f16"))
    b2 = gaussian_source(dims2, 154, 8)
    from paper_1010_4782_amd._lib import lib
    xs, infos = cg_solve_batch([(lat, bt, masses, None), (lat2, torch.from_numpy(b2).cuda(), 0.1, None)], tol=1e-10,
                               prec="f16", autotune=True)
    assert all(i["converged"] == 1 for i in infos)
    x2b = xs[1].cpu().numpy()
    for r in range(8):
        assert true_residual(lambda v: apply_m(fat2, lng2, v, dims2, 0.1), b2[r], x2b[r]) <= 1.05e-10


@pytest.mark.parametrize("long_su3", [True, False])
def test_dslash_f16_subnormal_site_scales(gpu_lib, long_su3):
    """An FP16 input scaled into binary32's subnormal range, as the edge of a point source's support is
    after a dozen CG iterations (site scales near 1e-39, whose reciprocal overflows): every output is
    finite and equals the unscaled result scaled down, to the precision subnormal scales keep, in the
    site-parallel and the time-streaming launches, which agree bit for bit."""
    dims = (8, 8, 8, 8)
    print(f"dslash f16 subnormal scales long_su3={long_su3}", flush=True)
    lat, fat, lng = make12(dims, 151, ("f64", "f16")) if long_su3 else make(dims, seed=151, precs=("f64", "f16"))
    b = gaussian_source(dims, 152, 8)
    sc = 2.0 ** -133
    bt, bs = torch.from_numpy(b).cuda(), torch.from_numpy(b * sc).cuda()
    for par in (0, 1):
        ref = lat.dslash(bt, par, prec="f16").cpu().numpy()
        outs = []
        for shape in ((64, 8, 0, 0), (64, 8, 0, 2, 1)):
            lat.set_dslash_shape("f16", 8, *shape)
            out = lat.dslash(bs, par, prec="f16").cpu().numpy()
            assert np.all(np.isfinite(out.real)) and np.all(np.isfinite(out.imag)), shape
            assert np.max(np.abs(out)) < 2.0 ** -126  # the output scales are subnormal
            assert rel(out / sc, ref) <= 1e-3, (par, shape)
            outs.append(out)
        assert np.array_equal(outs[0], outs[1]), par
    lat.set_dslash_shape("f16", 8, 0, 1)
