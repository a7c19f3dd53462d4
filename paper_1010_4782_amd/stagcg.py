"""Python binding of libstagcg.so: the same entry points as include/stagcg.h, taking torch tensors.

torch supplies device memory and the HIP stream; every step of the operator and
the solvers runs in the library's kernels.  Tensors are complex128 on the GPU:
links [4][Lt][Lz][Ly][Lx][3][3], even-odd vectors [nrhs][V/2][3] (or [V/2][3]).
"""
from __future__ import annotations

import ctypes as C
from typing import Iterable, Sequence

import torch

from . import _lib
from ._lib import (PREC, StagError, StagInfo, StagParams, StagProblem, StagShape, StagTrainInfo, StagTrainParams,
                   check, lib)

__all__ = ["Lattice", "Net", "cg_solve_batch", "StagError", "solve_params", "tune_cache_save", "tune_cache_load"]


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _dev_tensor(t: torch.Tensor, name: str, shape_tail=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != torch.complex128:
        raise TypeError(f"{name} must be complex128")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[-len(shape_tail):]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected [..., {shape_tail}]")
    return t


def solve_params(tol=1e-10, prec="f64", max_iter=0, reliable_interval=50, reliable_delta=0.1, check_interval=16,
                 max_restarts=5, profile=False, history_len=0, history=None, stall_window=10,
                 stall_ratio=0.9, autotune=False, net=None) -> StagParams:
    p = _lib.default_params()
    p.tol = tol
    p.prec = PREC[prec]
    p.max_iter = max_iter
    p.reliable_interval = reliable_interval
    p.reliable_delta = reliable_delta
    p.check_interval = check_interval
    p.max_restarts = max_restarts
    # profile: False/0 off, True = every iteration, k > 1 = every k-th iteration
    p.profile = int(profile) if not isinstance(profile, bool) else (1 if profile else 0)
    p.history_len = history_len
    if history is not None:
        p.history = history.ctypes.data_as(C.POINTER(C.c_double))
    p.stall_window = stall_window
    p.stall_ratio = stall_ratio
    p.autotune = 1 if autotune else 0
    if net is not None:
        p.precond = 1
        p.net = net.handle
    return p


def tune_cache_save(path: str):
    check(lib().stag_tune_cache_save(path.encode()), "stag_tune_cache_save")


def tune_cache_load(path: str):
    check(lib().stag_tune_cache_load(path.encode()), "stag_tune_cache_load")


class Lattice:
    """A lattice of extents (Lx, Ly, Lz, Lt) on the current GPU, with packed links once loaded."""

    def __init__(self, dims: Sequence[int], antiperiodic_t: bool = True):
        self.dims = tuple(int(d) for d in dims)
        h = C.c_void_p()
        arr = (C.c_int32 * 4)(*self.dims)
        check(lib().stag_create_lattice(arr, 1 if antiperiodic_t else 0, C.byref(h)), "stag_create_lattice")
        self._h = h
        self.half = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3] // 2
        self._keep = []

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            torch.cuda.synchronize()
            check(lib().stag_destroy_lattice(self._h), "stag_destroy_lattice")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, t, name):
        _dev_tensor(t, name, (self.half, 3))
        nrhs = 1 if t.dim() == 2 else int(t.numel() // (self.half * 3))
        return nrhs

    def load_links(self, fat: torch.Tensor, lng: torch.Tensor | None = None, naik: float = -1.0 / 24.0,
                   precs: Iterable[str] = ("f64",), long_su3: bool = False, stream=None):
        """Pack the links; long_su3=True stores the (SU(3)) three-hop links with 12 real parameters."""
        Lx, Ly, Lz, Lt = self.dims
        shape = (4, Lt, Lz, Ly, Lx, 3, 3)
        _dev_tensor(fat, "fat")
        if tuple(fat.shape) != shape:
            raise ValueError(f"fat links must have shape {shape}")
        if lng is not None:
            _dev_tensor(lng, "lng")
            if tuple(lng.shape) != shape:
                raise ValueError(f"long links must have shape {shape}")
        mask = 0x100 if long_su3 else 0
        for p in precs:
            mask |= 1 << PREC[p]
        check(lib().stag_load_links(self._h, fat.data_ptr(), None if lng is None else lng.data_ptr(), float(naik),
                                    mask, _stream(stream)), "stag_load_links")

    def fatten_links(self, thin: torch.Tensor, u0: float = 1.0, fat=None, lng=None, stream=None):
        """Asqtad one-hop links and three-hop products of a thin gauge field (stag_fatten_links); returns
        (fat, lng), each complex128 [4][Lt][Lz][Ly][Lx][3][3] on the device."""
        Lx, Ly, Lz, Lt = self.dims
        shape = (4, Lt, Lz, Ly, Lx, 3, 3)
        _dev_tensor(thin, "thin")
        if tuple(thin.shape) != shape:
            raise ValueError(f"thin links must have shape {shape}")
        fat = torch.empty_like(thin) if fat is None else fat
        lng = torch.empty_like(thin) if lng is None else lng
        for name, t in (("fat", fat), ("lng", lng)):
            _dev_tensor(t, name)
            if tuple(t.shape) != shape:
                raise ValueError(f"{name} must have shape {shape}")
        check(lib().stag_fatten_links(self._h, thin.data_ptr(), float(u0), fat.data_ptr(), lng.data_ptr(),
                                      _stream(stream)), "stag_fatten_links")
        return fat, lng

    def dslash(self, x: torch.Tensor, out_parity: int, prec: str = "f64", out=None, stream=None) -> torch.Tensor:
        nrhs = self._vec(x, "in")
        out = torch.empty_like(x) if out is None else out
        self._vec(out, "out")
        check(lib().stag_dslash(self._h, int(out_parity), x.data_ptr(), out.data_ptr(), nrhs, PREC[prec],
                                _stream(stream)), "stag_dslash")
        return out

    def dslash_slab(self, x_ext: torch.Tensor, out_parity: int, t0: int, lt: int, prec: str = "f64", out=None,
                    stream=None) -> torch.Tensor:
        """D on the time slab [t0, t0 + lt) from an extended input [nrhs][(lt + 6) S][3] (3 ghost slices
        on each side, S sites per slice and parity); returns [nrhs][lt S][3]."""
        S = self.half // self.dims[3]
        if x_ext.dim() == 2:
            x_ext = x_ext.unsqueeze(0)
        if x_ext.dtype != torch.complex128 or not x_ext.is_cuda or not x_ext.is_contiguous():
            raise ValueError("x_ext must be a contiguous complex128 CUDA tensor")
        if x_ext.shape[1:] != (int((lt + 6) * S), 3):
            raise ValueError(f"x_ext has shape {tuple(x_ext.shape)}, expected [nrhs, {(lt + 6) * S}, 3]")
        nrhs = x_ext.shape[0]
        out = torch.empty((nrhs, lt * S, 3), dtype=torch.complex128, device=x_ext.device) if out is None else out
        check(lib().stag_dslash_slab(self._h, int(out_parity), int(t0), int(lt), x_ext.data_ptr(), out.data_ptr(),
                                     nrhs, PREC[prec], _stream(stream)), "stag_dslash_slab")
        return out

    def slice_norm2(self, v: torch.Tensor, group: int = 1, weight: float = 1.0, out=None, accumulate=False,
                    stream=None) -> torch.Tensor:
        """out[g][t] (+)= weight * sum of |v|^2 over time slice t and the RHS of group g (float64 [n/group][Lt])."""
        nrhs = self._vec(v, "v")
        if nrhs % group:
            raise ValueError("group must divide the number of right-hand sides")
        if out is None:
            if accumulate:
                raise ValueError("accumulate needs out")
            out = torch.empty((nrhs // group, self.dims[3]), dtype=torch.float64, device=v.device)
        if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or \
                tuple(out.shape) != (nrhs // group, self.dims[3]):
            raise ValueError(f"out must be a contiguous float64 CUDA tensor of shape {(nrhs // group, self.dims[3])}")
        check(lib().stag_slice_norm2(self._h, v.data_ptr(), nrhs, int(group), float(weight), 1 if accumulate else 0,
                                     out.data_ptr(), _stream(stream)), "stag_slice_norm2")
        return out

    def pion_correlator(self, chi: torch.Tensor, mass: float, out=None, stream=None) -> torch.Tensor:
        """C[s][t] of point-source propagators from their even-site solutions chi (3 consecutive RHS, the
        source colours, per source), computed by stag_pion_correlator."""
        nrhs = self._vec(chi, "chi")
        if nrhs % 3:
            raise ValueError("chi holds three right-hand sides (source colours) per source")
        nsrc = nrhs // 3
        if out is None:
            out = torch.empty((nsrc, self.dims[3]), dtype=torch.float64, device=chi.device)
        if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or \
                tuple(out.shape) != (nsrc, self.dims[3]):
            raise ValueError(f"out must be a contiguous float64 CUDA tensor of shape {(nsrc, self.dims[3])}")
        check(lib().stag_pion_correlator(self._h, chi.data_ptr(), nsrc, float(mass), out.data_ptr(),
                                         _stream(stream)), "stag_pion_correlator")
        return out

    def apply_m(self, x: torch.Tensor, mass, out=None, stream=None) -> torch.Tensor:
        nrhs = self._vec(x, "in")
        masses = [float(mass)] * nrhs if not isinstance(mass, (list, tuple)) else [float(m) for m in mass]
        if len(masses) != nrhs:
            raise ValueError("one mass per right-hand side")
        out = torch.empty_like(x) if out is None else out
        self._vec(out, "out")
        m = (C.c_double * nrhs)(*masses)
        check(lib().stag_apply_m(self._h, m, x.data_ptr(), out.data_ptr(), nrhs, _stream(stream)), "stag_apply_m")
        return out

    def apply_m_noalloc(self, x: torch.Tensor, mass, out: torch.Tensor, stream=None) -> torch.Tensor:
        """M x through stag_apply_m_noalloc: the library allocates nothing (the caller passes `out`)."""
        nrhs = self._vec(x, "in")
        masses = [float(mass)] * nrhs if not isinstance(mass, (list, tuple)) else [float(m) for m in mass]
        if len(masses) != nrhs:
            raise ValueError("one mass per right-hand side")
        self._vec(out, "out")
        m = (C.c_double * nrhs)(*masses)
        check(lib().stag_apply_m_noalloc(self._h, m, x.data_ptr(), out.data_ptr(), nrhs, _stream(stream)),
              "stag_apply_m_noalloc")
        return out

    def tune_dslash(self, prec: str = "f64", nrhs: int = 1, stream=None):
        """Time every Dslash launch shape; returns (best, [(wg, rhs_per_lane, lds_stage, tile_order, t_chunks, us),
        ...])."""
        best = StagShape()
        all_ = (StagShape * 128)()
        n = C.c_int32(0)
        check(lib().stag_tune_dslash(self._h, PREC[prec], int(nrhs), C.byref(best), all_, 128, C.byref(n),
                                     _stream(stream)), "stag_tune_dslash")
        def tup(s):
            return (s.wg, s.rhs_per_lane, s.lds_stage, s.tile_order, s.t_chunks, s.us)

        return tup(best), [tup(all_[i]) for i in range(n.value)]

    def set_dslash_shape(self, prec: str, nrhs: int, wg: int, rhs_per_lane: int = 1, lds_stage: int = 0,
                         tile_order: int = 0, t_chunks: int = 1):
        """Pin a Dslash launch shape for (this lattice, nrhs, prec); wg = 0 removes the pinned shape."""
        sh = StagShape(int(wg), int(rhs_per_lane), int(lds_stage), int(tile_order), int(t_chunks), 0.0)
        check(lib().stag_set_dslash_shape(self._h, PREC[prec], int(nrhs), C.byref(sh) if wg else None),
              "stag_set_dslash_shape")

    def cg_solve(self, b: torch.Tensor, mass, x0: torch.Tensor | None = None, raise_on_fail=True, stream=None,
                 **params):
        """Solve (4m^2 - D_eo D_oe) x = b; returns (x, [info dict per RHS])."""
        nrhs = self._vec(b, "b")
        masses = [float(mass)] * nrhs if not isinstance(mass, (list, tuple)) else [float(m) for m in mass]
        if len(masses) != nrhs:
            raise ValueError("one mass per right-hand side")
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        prm = solve_params(**params)
        infos = (StagInfo * nrhs)()
        m = (C.c_double * nrhs)(*masses)
        st = lib().stag_cg_solve(self._h, m, b.data_ptr(), x.data_ptr(), nrhs, C.byref(prm), infos, _stream(stream))
        if raise_on_fail:
            check(st, "stag_cg_solve")
        return x, [i.as_dict() for i in infos]


def cg_solve_batch(problems, raise_on_fail=True, stream=None, **params):
    """problems: list of (Lattice, b, masses, x0 or None).  Returns ([x], [info dict per RHS in order])."""
    n = len(problems)
    arr = (StagProblem * n)()
    xs, keep = [], []
    total = 0
    for i, (lat, b, masses, x0) in enumerate(problems):
        nrhs = lat._vec(b, "b")
        masses = [float(masses)] * nrhs if not isinstance(masses, (list, tuple)) else [float(m) for m in masses]
        if len(masses) != nrhs:
            raise ValueError("one mass per right-hand side")
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        m = (C.c_double * nrhs)(*masses)
        keep.append(m)
        arr[i] = StagProblem(lat.handle, nrhs, C.cast(m, C.POINTER(C.c_double)), b.data_ptr(), x.data_ptr())
        xs.append(x)
        total += nrhs
    prm = solve_params(**params)
    infos = (StagInfo * total)()
    st = lib().stag_cg_solve_batch(n, arr, C.byref(prm), infos, _stream(stream))
    if raise_on_fail:
        check(st, "stag_cg_solve_batch")
    return xs, [i.as_dict() for i in infos]


class Net:
    """The gauge-covariant network preconditioner on a lattice (its FP32 links must be loaded)."""

    def __init__(self, lat: Lattice, layers: int = 4, channels: int = 8, seed: int = 0, hermitian: bool = False):
        h = C.c_void_p()
        check(lib().stag_net_create(lat.handle, int(layers), int(channels), 1 if hermitian else 0, int(seed),
                                    C.byref(h)), "stag_net_create")
        self.hermitian = hermitian
        self._h = h
        self.lat = lat
        self.layers = layers
        self.channels = channels
        self.ch = [1] + [channels] * (layers - 1) + [1] if layers > 1 else [1, 1]

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            torch.cuda.synchronize()
            check(lib().stag_net_destroy(self._h), "stag_net_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_weights(self) -> int:
        n = C.c_int64()
        check(lib().stag_net_num_weights(self._h, C.byref(n)), "stag_net_num_weights")
        return n.value

    def _flat(self, weights):
        import numpy as np

        flat = np.concatenate([np.asarray(w, dtype=np.complex128).reshape(-1) for w in weights])
        return np.ascontiguousarray(flat.view(np.float64))

    def _split(self, flat):
        import numpy as np

        z = flat.view(np.complex128)
        out, k = [], 0
        for ci, co in zip(self.ch[:-1], self.ch[1:]):
            n = 9 * co * ci
            out.append(z[k:k + n].reshape(9, co, ci).copy())
            k += n
        return out

    def set_weights(self, weights):
        flat = self._flat(weights)
        check(lib().stag_net_set_weights(self._h, flat.ctypes.data_as(C.POINTER(C.c_double)), flat.size // 2),
              "stag_net_set_weights")

    def get_weights(self):
        import numpy as np

        flat = np.zeros(2 * self.num_weights())
        check(lib().stag_net_get_weights(self._h, flat.ctypes.data_as(C.POINTER(C.c_double)), flat.size // 2),
              "stag_net_get_weights")
        return self._split(flat)

    def apply(self, r: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        nrhs = self.lat._vec(r, "in")
        out = torch.empty_like(r) if out is None else out
        check(lib().stag_net_apply(self._h, r.data_ptr(), out.data_ptr(), nrhs, _stream(stream)), "stag_net_apply")
        return out

    LOSS = {"solution": 0, "residual": 1}

    def loss_grad(self, b: torch.Tensor, x: torch.Tensor, loss="solution", mass=0.0, stream=None):
        import numpy as np

        n = self.lat._vec(b, "b")
        self.lat._vec(x, "x")
        val = C.c_double()
        g = np.zeros(2 * self.num_weights())
        check(lib().stag_net_loss_grad(self._h, b.data_ptr(), x.data_ptr(), n, self.LOSS[loss], float(mass),
                                       C.byref(val), g.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)),
              "stag_net_loss_grad")
        return val.value, self._split(g)

    def train(self, b: torch.Tensor, x: torch.Tensor, epochs=10, batch=8, lr=1e-3, seed=1, loss="residual", mass=0.0,
              stream=None) -> dict:
        n = self.lat._vec(b, "b")
        self.lat._vec(x, "x")
        p = StagTrainParams()
        lib().stag_train_params_default(C.byref(p))
        p.epochs, p.batch, p.lr, p.seed = int(epochs), int(batch), float(lr), int(seed)
        p.loss_kind, p.mass = self.LOSS[loss], float(mass)
        info = StagTrainInfo()
        check(lib().stag_net_train(self._h, b.data_ptr(), x.data_ptr(), n, C.byref(p), C.byref(info),
                                   _stream(stream)), "stag_net_train")
        return {k: getattr(info, k) for k, _ in info._fields_}
