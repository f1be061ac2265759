"""Python binding of libdmrg.so (MI355X DMRG sigma / renormalization / TDA).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device arrays are torch tensors (float64, on the context's GPU);
torch supplies device memory and the stream, nothing else.  The library must
be built first (``python -m paper_1311_1646_amd.build``); importing this module
without it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DMRG_LIBRARY selects another build of the same library (the host-sanitizer
# build, libdmrg_san.so, loaded with the sanitizer runtime preloaded)
LIB_PATH = os.environ.get("DMRG_LIBRARY") or os.path.join(_HERE, "libdmrg.so")

FP64, FP32, BF16X3 = 0, 1, 2
SIGMA_ZEROTH_1SITE, SIGMA_ZEROTH_2SITE, SIGMA_TDA_FULL, SIGMA_TDA_DH_LEFT = 0, 1, 2, 3
ZEROTH, FIRST = 0, 1
TDA_HIST = 256  # DMRG_TDA_HIST
DIR_LEFT, DIR_RIGHT = 0, 1

_ERRORS = {
    -1: "INVALID_ARG", -2: "OOM", -3: "NOT_CONVERGED", -4: "SINGULAR",
    -5: "HIP_ERROR", -6: "STATE", -7: "INTERNAL",
}


class DMRGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


# torch is imported before the library so that both resolve the HIP runtime
# (libamdhip64.so.7) to the same loaded copy; two runtimes in one process do
# not see the same devices.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1311_1646_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_IP = ctypes.POINTER(ctypes.c_int)
_DP = ctypes.POINTER(ctypes.c_double)
_SP = ctypes.POINTER(ctypes.c_size_t)


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "sigma_flops", "sigma_ms", "sigma_main_ms", "sigma_main_flops", "sigma_main_bytes",
        "renorm_flops", "renorm_ms", "op_bytes", "tda_iter_ms", "tda_sigma_flops")] + [
        ("tda_iters", ctypes.c_int), ("sigma_main_launches", ctypes.c_int), ("tda_sigma_ms", ctypes.c_double),
        ("plan_ms", ctypes.c_double), ("sigma_workspace_bytes", ctypes.c_double),
        ("tda_polish_iters", ctypes.c_int), ("tda_hist_len", ctypes.c_int),
        ("tda_r2_hist", ctypes.c_double * TDA_HIST), ("tda_total_ms", ctypes.c_double),
        ("tda_space", ctypes.c_int), ("tda_phase_ms", ctypes.c_double * 6)]


class SweepParams(ctypes.Structure):
    _fields_ = [("nsweeps", _I), ("M_schedule", _IP), ("noise", _DP), ("davidson_tol", _D),
                ("davidson_max_iter", _I), ("seed", _I), ("prec", _I), ("verbose", _I), ("onesite_sweeps", _I)]


class DavidsonParams(ctypes.Structure):
    _fields_ = [("max_iter", _I), ("max_space", _I), ("tol", _D), ("seed", _I), ("prec", _I),
                ("verbose", _I), ("polish", _I), ("guess", _I)]


def _sig(name, *args):
    f = getattr(_lib, name)
    f.argtypes = list(args)
    f.restype = _I
    return f


_create = _sig("dmrg_create", _I, _I, _I, _DP, _DP, _D, _I, _P, _P, ctypes.POINTER(_P))
_destroy = _sig("dmrg_destroy", _P)
_lib.dmrg_last_error.argtypes = [_P]
_lib.dmrg_last_error.restype = ctypes.c_char_p
_num_channels = _sig("dmrg_num_channels", _P, _I, _IP)
_import = _sig("dmrg_import_mps", _P, _IP, _IP, _DP, _DP, _DP, _DP)
_export = _sig("dmrg_export_mps", _P, _IP, _IP, _DP, _DP, _DP, _DP, _SP)
_layout = _sig("dmrg_get_layout", _P, _I, _I, _IP, _IP, _SP)
_build_ops = _sig("dmrg_build_ops", _P, _I)
_Z = ctypes.c_size_t
_sigma = _sig("dmrg_sigma", _P, _I, _I, _I, _P, _P, _Z, _I)
_diag = _sig("dmrg_diag", _P, _I, _I, _P, _Z, _I)
_sigma_noalloc = _sig("dmrg_sigma_noalloc", _P, _I, _I, _I, _P, _P, _Z, _I)
_autotune = _sig("dmrg_autotune", _P, _I, _I, _I, _IP, _DP)
_renorm = _sig("dmrg_renormalize", _P, _I, _I, _I, _I, _P, _Z, _I)
_sweep = _sig("dmrg_sweep_ground", _P, ctypes.POINTER(SweepParams), _DP, _DP)
_tda = _sig("dmrg_tda_roots", _P, _I, ctypes.POINTER(DavidsonParams), _DP, _DP, _DP, _IP)
_rpa = _sig("dmrg_rpa_roots", _P, _I, ctypes.POINTER(DavidsonParams), _DP, _DP, _DP, _IP)
_rpa_reduced = _sig("dmrg_rpa_reduced", _I, _DP, _DP, _DP, _D, _I, _DP, _DP, _DP)
_stats = _sig("dmrg_get_stats", _P, ctypes.POINTER(Stats))
_stats_size = _lib.dmrg_stats_size
_stats_size.argtypes = []
_stats_size.restype = ctypes.c_size_t
if _stats_size() != ctypes.sizeof(Stats):
    raise ImportError(f"dmrg_stats layout mismatch: library {_stats_size()} bytes, binding {ctypes.sizeof(Stats)}")
_tda_reduced = _sig("dmrg_tda_reduced", _P, _IP, _DP, _DP)
_response = _sig("dmrg_response", _P, _DP, _D, ctypes.POINTER(DavidsonParams), _DP, _DP, _IP)
_tda_transition = _sig("dmrg_tda_transition", _P, _I, ctypes.POINTER(DavidsonParams), _DP, _DP, _DP, _IP, _DP)
_debug_dense = _sig("dmrg_debug_mpo_dense", _P, _I, _I, _DP)
_group_create = _sig("dmrg_group_create", _P, _I, _IP, _I, _I, ctypes.POINTER(_P))
_group_sigma = _sig("dmrg_group_sigma", _P, _P, _P, _SP, _I)
_group_stats = _sig("dmrg_group_stats", _P, _DP, _DP, _IP, _IP)
_group_destroy = _sig("dmrg_group_destroy", _P)
_lib.dmrg_group_last_error.argtypes = [_P]
_lib.dmrg_group_last_error.restype = ctypes.c_char_p


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


def _torch_allocator(device):
    """dmrg_allocator backed by torch's caching allocator: the library's
    device memory (operator pools, MPS tensors, plans, workspaces) is then
    owned and recycled by torch, in stream order on the context's stream."""
    import torch

    def alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream or 0)
        except Exception:  # out of memory: the library reports DMRG_ERR_OOM
            return None

    def free(ptr, user):
        if ptr:
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:  # interpreter shutdown: torch's pool is already gone
                pass

    return Allocator(_ALLOC_FN(alloc), _FREE_FN(free), None)


def _dp(a):
    return a.ctypes.data_as(_DP)


def _ip(a):
    return a.ctypes.data_as(_IP)


def rpa_reduced(HR, SR, WR, e0, nroots):
    """The reduced DMRG-RPA problem alone, on the host (see dmrg_rpa_reduced):
    returns (omega[nroots], a, b, rank) with a, b of shape (l, nroots)."""
    HR, SR, WR = (np.ascontiguousarray(m, dtype=np.float64) for m in (HR, SR, WR))
    l = HR.shape[0]
    if HR.shape != (l, l) or SR.shape != (l, l) or WR.shape != (l, l):
        raise ValueError("HR, SR, WR must be square and of one size")
    om = np.zeros(nroots)
    a = np.zeros((nroots, l))
    b = np.zeros((nroots, l))
    rc = _rpa_reduced(l, _dp(HR), _dp(SR), _dp(WR), float(e0), nroots, _dp(om), _dp(a), _dp(b))
    if rc < 0:
        raise DMRGError(rc, "dmrg_rpa_reduced failed")
    return om, a.T.copy(), b.T.copy(), rc


class Context:
    """One problem (integrals, electron numbers) on one GPU (device >= 0) or
    host-only (device < 0: layout and test-support calls only)."""

    def __init__(self, L, n_alpha, n_beta, h, eri, ecore=0.0, device=0, stream=None, allocator="torch"):
        """allocator: "torch" (device memory from torch's caching allocator)
        or "hip" (the library's own hipMalloc / hipFree)."""
        self.L, self.na, self.nb = L, n_alpha, n_beta
        h = np.ascontiguousarray(h, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        if h.shape != (L, L) or eri.shape != (L, L, L, L):
            raise ValueError(f"integrals must have shapes ({L}, {L}) and ({L},) * 4")
        if allocator not in ("torch", "hip"):
            raise ValueError("allocator must be 'torch' or 'hip'")
        if stream is None and device >= 0:
            import torch
            torch.cuda.set_device(device)
            stream = torch.cuda.current_stream(device).cuda_stream
        self.device = device
        self._sizes = {}
        self._alloc = _torch_allocator(device) if (allocator == "torch" and device >= 0) else None
        self._h = ctypes.c_void_p()
        rc = _create(L, n_alpha, n_beta, _dp(h), _dp(eri), float(ecore), device,
                     ctypes.c_void_p(stream or 0),
                     ctypes.cast(ctypes.pointer(self._alloc), _P) if self._alloc is not None else None,
                     ctypes.byref(self._h))
        if rc != 0:
            raise DMRGError(rc, _lib.dmrg_last_error(None).decode())

    def _check(self, rc):
        if rc != 0:
            raise DMRGError(rc, _lib.dmrg_last_error(self._h).decode())

    def close(self):
        if self._h:
            if self._alloc is not None:
                import torch
                torch.cuda.synchronize(self.device)  # freed blocks go back to torch's pool
            _destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- structure
    def num_channels(self, bond):
        out = ctypes.c_int()
        self._check(_num_channels(self._h, bond, ctypes.byref(out)))
        return out.value

    def import_mps(self, nsec, sectors, Ldata, Rdata, Cdata, lam):
        nsec = np.ascontiguousarray(nsec, np.int32)
        sectors = np.ascontiguousarray(sectors, np.int32)
        arrs = [np.ascontiguousarray(a, np.float64) for a in (Ldata, Rdata, Cdata, lam)]
        self._check(_import(self._h, _ip(nsec), _ip(sectors), *[_dp(a) for a in arrs]))
        self._sizes = {}

    def export_mps(self):
        nsec = np.zeros(self.L + 1, np.int32)
        sizes = np.zeros(4, np.uint64)
        self._check(_export(self._h, _ip(nsec), None, None, None, None, None,
                            sizes.ctypes.data_as(_SP)))
        sec = np.zeros(3 * int(sizes[0]), np.int32)
        Ld = np.zeros(int(sizes[1]))
        Rd = np.zeros(int(sizes[1]))
        Cd = np.zeros(int(sizes[1]))
        lam = np.zeros(int(sizes[3]))
        self._check(_export(self._h, _ip(nsec), _ip(sec), _dp(Ld), _dp(Rd), _dp(Cd), _dp(lam),
                            sizes.ctypes.data_as(_SP)))
        return nsec, sec.reshape(-1, 3), Ld, Rd, Cd, lam

    def layout(self, site, width=1):
        nb = ctypes.c_int()
        size = ctypes.c_size_t()
        self._check(_layout(self._h, site, width, ctypes.byref(nb), None, ctypes.byref(size)))
        blocks = np.zeros(6 * nb.value, np.int32)
        self._check(_layout(self._h, site, width, ctypes.byref(nb), _ip(blocks), ctypes.byref(size)))
        return blocks.reshape(-1, 6), size.value

    def size(self, site, width=1):
        """Element count of the coefficient tensor at `site` (cached)."""
        key = (site, width)
        if key not in self._sizes:
            size = ctypes.c_size_t()
            self._check(_layout(self._h, site, width, None, None, ctypes.byref(size)))
            self._sizes[key] = size.value
        return self._sizes[key]

    def _vectors(self, name, t, size, nvec=None):
        """Check a device vector argument (float64, this context's GPU,
        contiguous, shape (size,) or (nvec, size)) and return its nvec."""
        import torch
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != torch.float64:
            raise ValueError(f"{name} must be float64, got {t.dtype}")
        if t.device != torch.device("cuda", self.device):
            raise ValueError(f"{name} must be on cuda:{self.device}, got {t.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.dim() not in (1, 2) or t.shape[-1] != size or t.numel() == 0:
            raise ValueError(f"{name} must have shape ({size},) or (nvec, {size}), got {tuple(t.shape)}")
        n = 1 if t.dim() == 1 else t.shape[0]
        if nvec is not None and n != nvec:
            raise ValueError(f"{name} holds {n} vectors, expected {nvec}")
        return n

    # ---- compute
    def build_ops(self, prec=FP64):
        self._check(_build_ops(self._h, prec))

    def sigma(self, site, C, kind=SIGMA_ZEROTH_1SITE, prec=FP64, out=None):
        """sigma = H_eff C (see dmrg_sigma).  C: float64 tensor on the
        context's GPU, (nvec, size) or (size,); out, when given, the same."""
        import torch
        width = 2 if kind == SIGMA_ZEROTH_2SITE else 1
        size = self.size(site, width)
        nvec = self._vectors("C", C, size)
        if out is None:
            out = torch.empty_like(C)
        else:
            self._vectors("out", out, size, nvec)
            if out.data_ptr() == C.data_ptr():
                raise ValueError("out must not alias C")
        self._check(_sigma(self._h, site, kind, nvec, ctypes.c_void_p(C.data_ptr()),
                           ctypes.c_void_p(out.data_ptr()), C.numel(), prec))
        return out

    def sigma_noalloc(self, site, C, out, kind=SIGMA_ZEROTH_1SITE, prec=FP64):
        """dmrg_sigma_noalloc: the zeroth-order sigma with workspaces from the
        library's static scratch; `out` must be given (nothing is allocated).
        Needs one sigma() call with the same site, kind, nvec and precision
        first."""
        width = 2 if kind == SIGMA_ZEROTH_2SITE else 1
        size = self.size(site, width)
        nvec = self._vectors("C", C, size)
        self._vectors("out", out, size, nvec)
        if out.data_ptr() == C.data_ptr():
            raise ValueError("out must not alias C")
        self._check(_sigma_noalloc(self._h, site, kind, nvec, ctypes.c_void_p(C.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), C.numel(), prec))
        return out

    def autotune(self, site, nvec, prec=FP32):
        """Pick the stage-1 / stage-2 tile shapes by timing the sigma at `site`
        (see dmrg_autotune); returns (stage1_shape, stage2_shape, best_ms)."""
        shapes = (ctypes.c_int * 2)()
        ms = ctypes.c_double()
        self._check(_autotune(self._h, site, nvec, prec, shapes, ctypes.byref(ms)))
        return shapes[0], shapes[1], ms.value

    def diag(self, site, width=1, prec=FP64):
        import torch
        size = self.size(site, width)
        out = torch.empty(size, dtype=torch.float64, device=f"cuda:{self.device}")
        self._check(_diag(self._h, site, width, ctypes.c_void_p(out.data_ptr()), size, prec))
        return out

    def renormalize(self, site, direction, order=ZEROTH, prec=FP64, A1=None):
        """order ZEROTH: recompute the zeroth-order operators across `site`.
        order FIRST: grow the first-order chain of `direction` by `site` with
        the first-order tensors A1 ((nvec, size) float64 on the GPU)."""
        if order == ZEROTH:
            if A1 is not None:
                raise ValueError("zeroth-order renormalization takes no tensors")
            self._check(_renorm(self._h, site, direction, order, 0, None, 0, prec))
            return
        nvec = self._vectors("A1", A1, self.size(site, 1))
        self._check(_renorm(self._h, site, direction, order, nvec, ctypes.c_void_p(A1.data_ptr()),
                            A1.numel(), prec))

    def sweep_ground(self, M_schedule, noise=None, davidson_tol=1e-12, davidson_max_iter=40,
                     seed=1, prec=FP64, verbose=0, onesite_sweeps=0):
        """Two-site sweeps with the bond schedule M_schedule, then
        onesite_sweeps one-site sweeps (see dmrg_sweep_ground); returns
        (energy, largest discarded weight of the last two-site sweep, True)."""
        Ms = np.ascontiguousarray(M_schedule, np.int32)
        nz = None if noise is None else np.ascontiguousarray(noise, np.float64)
        p = SweepParams(len(Ms), _ip(Ms), _dp(nz) if nz is not None else None, davidson_tol,
                        davidson_max_iter, seed, prec, verbose, int(onesite_sweeps))
        e = ctypes.c_double()
        dw = ctypes.c_double()
        rc = _sweep(self._h, ctypes.byref(p), ctypes.byref(e), ctypes.byref(dw))
        self._sizes = {}
        self._check(rc)
        return e.value, dw.value, True

    def tda_roots(self, nroots, max_iter=60, max_space=0, tol=1e-9, seed=7, prec=FP64, verbose=0, polish=True,
                  guess="diag"):
        """DMRG-TDA roots (see dmrg_tda_roots); polish: an FP32 or BF16X3 run
        ends with FP64 iterations (stats()["tda_polish_iters"] says how many); guess:
        "diag" (lowest diagonal elements at the middle site) or "random"."""
        if guess not in ("diag", "random"):
            raise ValueError("guess must be 'diag' or 'random'")
        p = DavidsonParams(max_iter, max_space, tol, seed, prec, verbose, 0 if polish else -1,
                           0 if guess == "diag" else 1)
        om = np.zeros(nroots)
        et = np.zeros(nroots)
        r2 = np.zeros(nroots)
        it = ctypes.c_int()
        if self._alloc is not None and max_space == 0:
            # the library sizes the trial space from the device's free memory:
            # hand torch's cached blocks back first so that they count as free
            import torch
            torch.cuda.synchronize(self.device)
            torch.cuda.empty_cache()
        rc = _tda(self._h, nroots, ctypes.byref(p), _dp(om), _dp(et), _dp(r2), ctypes.byref(it))
        if rc not in (0, -3):
            self._check(rc)
        return om, et, r2, it.value, rc == 0

    def rpa_roots(self, nroots, max_iter=60, max_space=0, tol=1e-9, seed=7, prec=FP64, verbose=0, polish=True,
                  guess="diag"):
        """DMRG-RPA roots (see dmrg_rpa_roots): returns (omega, e_total,
        resid2, iterations, converged)."""
        if guess not in ("diag", "random"):
            raise ValueError("guess must be 'diag' or 'random'")
        p = DavidsonParams(max_iter, max_space, tol, seed, prec, verbose, 0 if polish else -1,
                           0 if guess == "diag" else 1)
        om = np.zeros(nroots)
        et = np.zeros(nroots)
        r2 = np.zeros(nroots)
        it = ctypes.c_int()
        if self._alloc is not None and max_space == 0:
            import torch
            torch.cuda.synchronize(self.device)
            torch.cuda.empty_cache()
        rc = _rpa(self._h, nroots, ctypes.byref(p), _dp(om), _dp(et), _dp(r2), ctypes.byref(it))
        if rc not in (0, -3):
            self._check(rc)
        return om, et, r2, it.value, rc == 0

    def tda_transition(self, nroots, max_iter=60, max_space=0, tol=1e-9, seed=7, prec=FP64, verbose=0, polish=True,
                       guess="diag"):
        """DMRG-TDA roots and their transition densities (see
        dmrg_tda_transition): returns (omega, e_total, resid2, iterations,
        converged, gamma) with gamma[nu, p, q] = <Psi^nu | E_pq | Psi0>."""
        if guess not in ("diag", "random"):
            raise ValueError("guess must be 'diag' or 'random'")
        p = DavidsonParams(max_iter, max_space, tol, seed, prec, verbose, 0 if polish else -1,
                           0 if guess == "diag" else 1)
        om = np.zeros(nroots)
        et = np.zeros(nroots)
        r2 = np.zeros(nroots)
        gamma = np.zeros((nroots, self.L, self.L))
        it = ctypes.c_int()
        if self._alloc is not None and max_space == 0:
            import torch
            torch.cuda.synchronize(self.device)
            torch.cuda.empty_cache()
        rc = _tda_transition(self._h, nroots, ctypes.byref(p), _dp(om), _dp(et), _dp(r2), ctypes.byref(it),
                             _dp(gamma))
        if rc not in (0, -3):
            self._check(rc)
        return om, et, r2, it.value, rc == 0, gamma

    def response(self, v, omega, max_iter=80, max_space=0, tol=1e-10, prec=FP64, verbose=0, polish=True):
        """Linear response to the one-body perturbation V = sum_pq v_pq E_pq at
        frequency omega (see dmrg_response): returns (chi_plus, chi_minus,
        resid2, iterations, converged) with chi_pm = <V Psi0 | Psi1_pm>."""
        v = np.ascontiguousarray(v, dtype=np.float64)
        if v.shape != (self.L, self.L):
            raise ValueError(f"v must have shape ({self.L}, {self.L})")
        p = DavidsonParams(max_iter, max_space, tol, 0, prec, verbose, 0 if polish else -1, 0)
        chi = np.zeros(2)
        r2 = np.zeros(2)
        it = ctypes.c_int()
        if self._alloc is not None and max_space == 0:
            import torch
            torch.cuda.synchronize(self.device)
            torch.cuda.empty_cache()
        rc = _response(self._h, _dp(v), float(omega), ctypes.byref(p), _dp(chi), _dp(r2), ctypes.byref(it))
        if rc not in (0, -3):
            self._check(rc)
        return float(chi[0]), float(chi[1]), r2, it.value, rc == 0

    def tda_reduced(self):
        """(H_R, S_R) of the last TDA forward sweep (l x l numpy arrays)."""
        l = ctypes.c_int()
        self._check(_tda_reduced(self._h, ctypes.byref(l), None, None))
        HR = np.zeros((l.value, l.value))
        SR = np.zeros((l.value, l.value))
        self._check(_tda_reduced(self._h, ctypes.byref(l), _dp(HR), _dp(SR)))
        return HR, SR

    def stats(self):
        s = Stats()
        self._check(_stats(self._h, ctypes.byref(s)))
        out = {k: getattr(s, k) for k, _ in Stats._fields_}
        out["tda_r2_hist"] = list(s.tda_r2_hist[:s.tda_hist_len])
        out["tda_phase_ms"] = dict(zip(("sigma1", "sigma0", "ren11", "ren01", "vec", "host"), s.tda_phase_ms))
        return out

    def debug_mpo_dense(self, wide_bond=-1, from_right=False):
        out = np.zeros((4 ** self.L, 4 ** self.L))
        self._check(_debug_dense(self._h, wide_bond, int(from_right), _dp(out)))
        return out


class Group:
    """Grouped zeroth-order sigma of many independent contexts (see
    dmrg_group_create): one launch per contraction stage for all members,
    optionally replayed from a HIP graph.  Keeps its contexts alive; close()
    before closing them."""

    def __init__(self, contexts, sites, nvec, prec=FP32):
        self.ctx = list(contexts)
        self.sites = [int(x) for x in sites]
        if len(self.sites) != len(self.ctx):
            raise ValueError("one site per context")
        self.nvec, self.prec = int(nvec), prec
        self.sizes = [c.size(i) for c, i in zip(self.ctx, self.sites)]
        hs = (_P * len(self.ctx))(*[c._h.value for c in self.ctx])
        st = np.ascontiguousarray(self.sites, np.int32)
        self._h = ctypes.c_void_p()
        rc = _group_create(ctypes.cast(hs, _P), len(self.ctx), _ip(st), self.nvec, prec, ctypes.byref(self._h))
        if rc != 0:
            raise DMRGError(rc, _lib.dmrg_group_last_error(None).decode())

    def _check(self, rc):
        if rc != 0:
            raise DMRGError(rc, _lib.dmrg_group_last_error(self._h).decode())

    def sigma(self, Cs, outs, graph=True):
        """One step: outs[i] = H_eff(member i) Cs[i]; each a float64 (nvec,
        size_i) tensor on the members' GPU."""
        n = len(self.ctx)
        if len(Cs) != n or len(outs) != n:
            raise ValueError(f"need {n} input and output tensors")
        for i, (c, C, O) in enumerate(zip(self.ctx, Cs, outs)):
            c._vectors(f"C[{i}]", C, self.sizes[i], self.nvec)
            c._vectors(f"out[{i}]", O, self.sizes[i], self.nvec)
        cp = (_P * n)(*[C.data_ptr() for C in Cs])
        op = (_P * n)(*[O.data_ptr() for O in outs])
        lens = (ctypes.c_size_t * n)(*[C.numel() for C in Cs])
        self._check(_group_sigma(self._h, ctypes.cast(cp, _P), ctypes.cast(op, _P), lens, int(bool(graph))))
        return outs

    def stats(self):
        fl, ms = ctypes.c_double(), ctypes.c_double()
        nl, nn = ctypes.c_int(), ctypes.c_int()
        self._check(_group_stats(self._h, ctypes.byref(fl), ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(nn)))
        return {"flops": fl.value, "ms": ms.value, "launches": nl.value, "graph_nodes": nn.value}

    def close(self):
        if self._h:
            _group_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
