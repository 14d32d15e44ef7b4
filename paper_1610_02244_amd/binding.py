"""ctypes binding of libtnt_mi355x.so (argument marshalling only).

Every computation runs in the HIP library; this module packs U(1) block
dicts into contiguous planes (torch device tensors supply the memory and the
stream), fills the C descriptors of include/tnt.h and unpacks results.
There is no fallback: without the built library, `load()` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libtnt_mi355x.so")

TNT_OK, TNT_W_NOCONV = 0, 1
TNT_FP64, TNT_FP32, TNT_BF16X3 = 0, 1, 2
TNT_DT_F64, TNT_DT_F32 = 0, 1
TNT_ABSORB_RIGHT, TNT_ABSORB_LEFT = 0, 1
TNT_ERR_2NORM, TNT_ERR_SUMSQ, TNT_ERR_1NORM = 0, 1, 2
PRECISIONS = {"fp64": TNT_FP64, "fp32": TNT_FP32, "bf16x3": TNT_BF16X3}

STATUS = {0: "TNT_OK", 1: "TNT_W_NOCONV", -1: "TNT_E_ARG", -2: "TNT_E_SHAPE",
          -3: "TNT_E_CHARGE", -4: "TNT_E_CAPACITY", -5: "TNT_E_ALLOC", -6: "TNT_E_NONFINITE",
          -7: "TNT_E_HIP", -8: "TNT_E_STATE"}

P = C.c_void_p
I32P = C.POINTER(C.c_int32)
I64P = C.POINTER(C.c_int64)
F64P = C.POINTER(C.c_double)


class BTensor(C.Structure):
    _fields_ = [("rank", C.c_int32), ("nblocks", C.c_int32), ("qn", I32P), ("extent", I32P),
                ("offset", I64P), ("re", P), ("im", P), ("dtype", C.c_int32),
                ("capacity", C.c_int64)]


class MpoSite(C.Structure):
    _fields_ = [("d", C.c_int32), ("D", C.c_int32), ("bond_charge", I32P), ("W", F64P)]


class LanczosParams(C.Structure):
    _fields_ = [("kmax", C.c_int32), ("precision", C.c_int32), ("beta_tol", C.c_double),
                ("resid_tol", C.c_double)]


class LanczosResult(C.Structure):
    _fields_ = [("E_ritz", C.c_double), ("E_refined", C.c_double), ("residual", C.c_double),
                ("steps", C.c_int32)]


class TruncParams(C.Structure):
    _fields_ = [("chi_max", C.c_int32), ("err_type", C.c_int32), ("abs_tol", C.c_double),
                ("rel_tol", C.c_double), ("err_tol", C.c_double), ("renormalise", C.c_int32)]


class SiteOut(C.Structure):
    _fields_ = [("max_blocks", C.c_int32), ("nblocks", C.c_int32), ("qn", I32P),
                ("extent", I32P), ("offset", I64P), ("re", F64P), ("im", F64P),
                ("capacity", C.c_int64)]


class TruncResult(C.Structure):
    _fields_ = [("chi", C.c_int32), ("nsectors", C.c_int32), ("eps", C.c_double),
                ("lambda0", C.c_double), ("norm_kept", C.c_double)]


class SweepParams(C.Structure):
    _fields_ = [("lanczos", LanczosParams), ("trunc", TruncParams), ("record_cap", C.c_int32),
                ("bond_E", F64P), ("bond_eps", F64P), ("bond_chi", I32P), ("bond_steps", I32P)]


class SweepResult(C.Structure):
    _fields_ = [("energy", C.c_double), ("max_residual", C.c_double), ("max_eps", C.c_double),
                ("updates", C.c_int32), ("max_chi", C.c_int32), ("matvecs", C.c_int64),
                ("matvec_flops", C.c_double), ("seconds_total", C.c_double),
                ("seconds_matvec", C.c_double), ("seconds_lanczos", C.c_double),
                ("seconds_svd", C.c_double), ("seconds_env", C.c_double),
                ("gemm_flops", C.c_double), ("seconds_gemm", C.c_double),
                ("gemm_launches", C.c_int64), ("seconds_theta", C.c_double),
                ("seconds_setup", C.c_double), ("eig_retries", C.c_int64)]


# name -> (restype, argtypes); mirrors include/tnt.h
SIGNATURES = {
    "tnt_ctx_create": (C.c_int32, [C.c_int32, P, C.POINTER(P)]),
    "tnt_ctx_destroy": (None, [P]),
    "tnt_last_error": (C.c_char_p, [P]),
    "tnt_sync": (C.c_int32, [P]),
    "tnt_pool_bytes": (C.c_int64, [P]),
    "tnt_ctx_memory": (C.c_int32, [P, C.POINTER(C.c_int64)]),
    "tnt_ctx_set_autotune": (C.c_int32, [P, C.c_int32]),
    "tnt_ctx_set_graphs": (C.c_int32, [P, C.c_int32]),
    "tnt_ctx_set_eig_reduction": (C.c_int32, [P, C.c_int32]),
    "tnt_mpo_spin1_heisenberg": (C.c_int32, [C.c_double, F64P, I32P]),
    "tnt_mpo_bose_hubbard": (C.c_int32, [C.c_int32, C.c_double, C.c_double, C.c_double, F64P,
                                         I32P]),
    "tnt_heff2_apply": (C.c_int32, [P, C.POINTER(BTensor), C.POINTER(MpoSite),
                                    C.POINTER(MpoSite), C.POINTER(BTensor),
                                    C.POINTER(BTensor), C.POINTER(BTensor), C.c_int32]),
    "tnt_heff2_apply_noalloc": (C.c_int32, [P, C.POINTER(BTensor), C.POINTER(MpoSite),
                                    C.POINTER(MpoSite), C.POINTER(BTensor),
                                    C.POINTER(BTensor), C.POINTER(BTensor), C.c_int32]),
    "tnt_heff2_flops": (C.c_int64, [C.POINTER(BTensor), C.POINTER(MpoSite), C.POINTER(MpoSite),
                                    C.POINTER(BTensor), C.POINTER(BTensor), I64P]),
    "tnt_lanczos_ground": (C.c_int32, [P, C.POINTER(BTensor), C.POINTER(MpoSite),
                                       C.POINTER(MpoSite), C.POINTER(BTensor),
                                       C.POINTER(BTensor), C.POINTER(LanczosParams),
                                       C.POINTER(LanczosResult)]),
    "tnt_theta_svd_truncate": (C.c_int32, [P, C.POINTER(BTensor), C.POINTER(TruncParams),
                                           C.c_int32, C.POINTER(SiteOut), C.POINTER(SiteOut),
                                           F64P, C.c_int32, I32P, I32P,
                                           C.POINTER(TruncResult)]),
    "tnt_trunc_select": (C.c_int32, [F64P, C.c_int32, C.POINTER(TruncParams), F64P]),
    "tnt_mps_create": (C.c_int32, [P, C.c_int32, C.c_int32, C.POINTER(P)]),
    "tnt_mps_destroy": (None, [P]),
    "tnt_mps_set_bond": (C.c_int32, [P, C.c_int32, C.c_int32, I32P, I32P]),
    "tnt_mps_set_site": (C.c_int32, [P, C.c_int32, C.c_int32, I32P, I32P, F64P, F64P]),
    "tnt_mps_bond_size": (C.c_int32, [P, C.c_int32]),
    "tnt_mps_get_bond": (C.c_int32, [P, C.c_int32, C.c_int32, I32P, I32P]),
    "tnt_mps_get_site": (C.c_int32, [P, C.c_int32, C.c_int32, I32P, I32P, I32P, C.c_int64,
                                     F64P, F64P]),
    "tnt_mps_right_canonicalize": (C.c_int32, [P, P]),
    "tnt_mps_correlation": (C.c_int32, [P, P, F64P, C.c_int32, F64P, F64P, F64P]),
    "tnt_heff1_apply": (C.c_int32, [P, P, P, P, P, P]),
    "tnt_auto_block_svd": (C.c_int32, [P, F64P, F64P, C.c_int32, C.c_int32, C.c_int64,
                                       C.c_double, P, F64P, F64P, C.c_int64, F64P, F64P,
                                       C.c_int64, F64P, I32P, I32P, F64P]),
    "tnt_tebd_step": (C.c_int32, [P, P, F64P, C.c_double, P, C.c_int32, F64P, I32P, F64P]),
    "tnt_bond_hamiltonians_bose_hubbard": (C.c_int32, [C.c_int32, C.c_int32, C.c_double,
                                                       C.c_double, C.c_double, F64P]),
    "tnt_bond_hamiltonians_spin1": (C.c_int32, [C.c_int32, C.c_double, F64P]),
    "tnt_env_create": (C.c_int32, [P, P, C.POINTER(MpoSite), C.c_int32, C.c_int32,
                                   C.POINTER(P)]),
    "tnt_env_destroy": (None, [P]),
    "tnt_dmrg_sweep": (C.c_int32, [P, P, P, C.POINTER(SweepParams), C.POINTER(SweepResult)]),
    "tnt_dmrg_sweep_batched": (C.c_int32, [P, C.c_int32, C.POINTER(P), C.POINTER(P),
                                           C.POINTER(SweepParams), C.POINTER(SweepResult)]),
    "tnt_heff2_apply_batched": (C.c_int32, [P, C.c_int32, C.POINTER(C.POINTER(BTensor)),
                                            C.POINTER(C.POINTER(MpoSite)),
                                            C.POINTER(C.POINTER(MpoSite)),
                                            C.POINTER(C.POINTER(BTensor)),
                                            C.POINTER(C.POINTER(BTensor)),
                                            C.POINTER(C.POINTER(BTensor)), C.c_int32]),
    "tnt_lanczos_ground_batched": (C.c_int32, [P, C.c_int32, C.POINTER(C.POINTER(BTensor)),
                                               C.POINTER(C.POINTER(MpoSite)),
                                               C.POINTER(C.POINTER(MpoSite)),
                                               C.POINTER(C.POINTER(BTensor)),
                                               C.POINTER(C.POINTER(BTensor)),
                                               C.POINTER(LanczosParams),
                                               C.POINTER(LanczosResult)]),
}


class TntError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} -> {STATUS.get(code, code)}: {msg}")
        self.code = code


def open_library(path: str = LIBPATH) -> C.CDLL:
    """Load the shared library and declare every exported signature."""
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(path)
    missing = []
    for name, (res, args) in SIGNATURES.items():
        try:
            fn = getattr(lib, name)
        except AttributeError:
            missing.append(name)
            continue
        fn.restype = res
        fn.argtypes = args
    lib.missing_symbols = missing
    return lib


MPO_LEFT, MPO_RIGHT = 3, 0  # boundary indices of the Bose-Hubbard MPO
SPIN1_LEFT, SPIN1_RIGHT = 4, 0  # boundary indices of the spin-1 Heisenberg MPO


def bose_hubbard_mpo(lib, nmax, J, U, mu=0.0):
    """(W[w, w', s', s], bond charges) from the library's MPO builder."""
    d = nmax + 1
    W = np.zeros((4, 4, d, d))
    qw = np.zeros(4, np.int32)
    code = lib.tnt_mpo_bose_hubbard(int(nmax), float(J), float(U), float(mu),
                                    W.ctypes.data_as(F64P), qw.ctypes.data_as(I32P))
    if code != 0:
        raise TntError("tnt_mpo_bose_hubbard", code, "invalid model parameters")
    return W, [int(x) for x in qw]


def spin1_heisenberg_mpo(lib, J):
    """(W[w, w', s', s], bond charges) of the spin-1 Heisenberg chain."""
    W = np.zeros((5, 5, 3, 3))
    qw = np.zeros(5, np.int32)
    code = lib.tnt_mpo_spin1_heisenberg(float(J), W.ctypes.data_as(F64P),
                                        qw.ctypes.data_as(I32P))
    if code != 0:
        raise TntError("tnt_mpo_spin1_heisenberg", code, "invalid model parameters")
    return W, [int(x) for x in qw]


def bond_hamiltonians_bose_hubbard(lib, L, nmax, J, U, mu=0.0):
    """(L-1, d^2, d^2) bond Hamiltonians of the Bose-Hubbard chain."""
    d = nmax + 1
    h = np.zeros((L - 1, d * d, d * d))
    code = lib.tnt_bond_hamiltonians_bose_hubbard(int(L), int(nmax), float(J), float(U),
                                                  float(mu), h.ctypes.data_as(F64P))
    if code != 0:
        raise TntError("tnt_bond_hamiltonians_bose_hubbard", code, "invalid model parameters")
    return h


def bond_hamiltonians_spin1(lib, L, J=1.0):
    h = np.zeros((L - 1, 9, 9))
    code = lib.tnt_bond_hamiltonians_spin1(int(L), float(J), h.ctypes.data_as(F64P))
    if code != 0:
        raise TntError("tnt_bond_hamiltonians_spin1", code, "invalid model parameters")
    return h


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _i64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _ptr(a, typ):
    return a.ctypes.data_as(typ)


class Descriptor:
    """A tnt_btensor plus the host arrays and device tensors it points at."""

    def __init__(self, rank, keys_qn, extents, offsets, re, im, dtype=TNT_DT_F64):
        self.qn = _i32(np.asarray(keys_qn).reshape(-1)) if len(keys_qn) else np.zeros(0, np.int32)
        self.ext = _i32(np.asarray(extents).reshape(-1)) if len(extents) else np.zeros(0, np.int32)
        self.off = _i64(offsets) if len(offsets) else np.zeros(0, np.int64)
        self.re, self.im = re, im
        cap = 0 if re is None else int(re.numel())
        self.c = BTensor(rank, len(offsets), _ptr(self.qn, I32P), _ptr(self.ext, I32P),
                         _ptr(self.off, I64P), P(re.data_ptr() if re is not None else 0),
                         P(im.data_ptr() if im is not None else 0), dtype, cap)

    @property
    def ref(self):
        return C.byref(self.c)


class Mpo:
    def __init__(self, W: np.ndarray, qw):
        self.W = np.ascontiguousarray(W, dtype=np.float64)
        self.qw = _i32(qw)
        D, _, d, _ = self.W.shape
        self.c = MpoSite(d, D, _ptr(self.qw, I32P), _ptr(self.W, F64P))

    @property
    def ref(self):
        return C.byref(self.c)


class Tnt:
    """A live library context bound to torch's current HIP stream on cuda:0."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the library runs on the GPU only")
        self.lib = open_library()
        self.device = device
        self.dev = torch.device("cuda", device)
        stream = torch.cuda.current_stream(self.dev).cuda_stream
        h = P()
        self._check("tnt_ctx_create", self.lib.tnt_ctx_create(device, P(stream), C.byref(h)), None)
        self.ctx = h

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.tnt_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, fn, code, ctx=-1):
        if code < 0:
            msg = ""
            c = self.ctx if ctx == -1 else ctx
            if c:
                msg = self.lib.tnt_last_error(c).decode()
            raise TntError(fn, code, msg)
        return code

    def bose_hubbard_mpo(self, nmax, J, U, mu=0.0):
        return bose_hubbard_mpo(self.lib, nmax, J, U, mu)

    def spin1_heisenberg_mpo(self, J=1.0):
        return spin1_heisenberg_mpo(self.lib, J)

    # -- packing helpers ----------------------------------------------------
    def planes(self, n, dtype=None):
        t = self.torch
        dt = t.float64 if dtype is None else dtype
        return t.zeros(max(n, 1), dtype=dt, device=self.dev), t.zeros(max(n, 1), dtype=dt,
                                                                      device=self.dev)

    def _upload(self, blocks_list):
        t = self.torch
        if blocks_list:
            flat = np.concatenate([b.reshape(-1) for b in blocks_list])
        else:
            flat = np.zeros(0, dtype=complex)
        re = t.from_numpy(np.ascontiguousarray(flat.real)).to(self.dev) if flat.size else \
            t.zeros(1, dtype=t.float64, device=self.dev)
        im = t.from_numpy(np.ascontiguousarray(flat.imag)).to(self.dev) if flat.size else \
            t.zeros(1, dtype=t.float64, device=self.dev)
        return re, im

    def theta(self, th: dict, keys=None):
        """Descriptor of a theta block dict {(q_a, s1, s2): (dim_a, dim_b)}."""
        keys = sorted(th) if keys is None else keys
        qn, ext, off, pos = [], [], [], 0
        for (qa, s1, s2) in keys:
            r, c = th[(qa, s1, s2)].shape
            qn.append((qa, s1, s2, qa + s1 + s2))
            ext.append((r, 1, 1, c))
            off.append(pos)
            pos += r * c
        re, im = self._upload([th[k] for k in keys])
        d = Descriptor(4, qn, ext, off, re, im)
        d.keys = keys
        d.shapes = [th[k].shape for k in keys]
        return d

    def site(self, A: dict, keys=None):
        """Descriptor of a site tensor {(q_a, s): (dim_a, dim_b)}."""
        keys = sorted(A) if keys is None else keys
        qn, ext, off, pos = [], [], [], 0
        for (qa, s) in keys:
            r, c = A[(qa, s)].shape
            qn.append((qa, s, qa + s))
            ext.append((r, 1, c))
            off.append(pos)
            pos += r * c
        re, im = self._upload([A[k] for k in keys])
        d = Descriptor(3, qn, ext, off, re, im)
        d.keys = keys
        d.shapes = [A[k].shape for k in keys]
        return d

    def site_like(self, desc: Descriptor):
        re, im = self.planes(int(desc.re.numel()))
        d = Descriptor(3, desc.qn.reshape(-1, 3), desc.ext.reshape(-1, 3), desc.off, re, im)
        d.keys, d.shapes = desc.keys, desc.shapes
        return d

    def heff1_apply(self, L, W, R, A, out):
        return self._check("tnt_heff1_apply",
                           self.lib.tnt_heff1_apply(self.ctx, L.ref, W.ref, R.ref, A.ref, out.ref))

    def theta_like(self, desc: Descriptor):
        re, im = self.planes(int(desc.re.numel()))
        d = Descriptor(4, desc.qn.reshape(-1, 4), desc.ext.reshape(-1, 4), desc.off, re, im)
        d.keys, d.shapes = desc.keys, desc.shapes
        return d

    def env(self, E: dict, qw):
        """Descriptor of an environment {(w, q): (dim(q + qw[w]), dim(q))}."""
        keys = sorted(E, key=lambda k: (k[1], k[0]))
        qn, ext, off, pos = [], [], [], 0
        for (w, q) in keys:
            r, c = E[(w, q)].shape
            qn.append((q + qw[w], w, q))
            ext.append((r, 1, c))
            off.append(pos)
            pos += r * c
        re, im = self._upload([E[k] for k in keys])
        return Descriptor(3, qn, ext, off, re, im)

    def download(self, desc: Descriptor) -> dict:
        self.sync()
        re = desc.re.detach().cpu().numpy()
        im = desc.im.detach().cpu().numpy()
        out = {}
        for k, shp, o in zip(desc.keys, desc.shapes, desc.off):
            n = shp[0] * shp[1]
            out[k] = (re[o:o + n] + 1j * im[o:o + n]).reshape(shp)
        return out

    # -- calls ----------------------------------------------------------------
    def sync(self):
        self._check("tnt_sync", self.lib.tnt_sync(self.ctx))

    def pool_bytes(self):
        return int(self.lib.tnt_pool_bytes(self.ctx))

    def memory(self) -> dict:
        """tnt_ctx_memory: the pool's held / in-use / peak in-use bytes and
        the rocBLAS / rocSOLVER handles' device workspace."""
        out = (C.c_int64 * 4)()
        self._check("tnt_ctx_memory", self.lib.tnt_ctx_memory(self.ctx, out))
        return {"pool_held": int(out[0]), "pool_in_use": int(out[1]),
                "pool_peak_in_use": int(out[2]), "blas_workspace": int(out[3])}

    def set_autotune(self, on: bool):
        self._check("tnt_ctx_set_autotune", self.lib.tnt_ctx_set_autotune(self.ctx, int(on)))

    def set_graphs(self, on: bool):
        self._check("tnt_ctx_set_graphs", self.lib.tnt_ctx_set_graphs(self.ctx, int(on)))

    def set_eig_reduction(self, min_order: int):
        """Padded sector order from which the SVD's eigenproblems use the
        library's own tridiagonal reduction (0: rocSOLVER's eigensolver for
        all; negative: the library default)."""
        self._check("tnt_ctx_set_eig_reduction",
                    self.lib.tnt_ctx_set_eig_reduction(self.ctx, int(min_order)))

    def heff2_apply(self, L, W1, W2, R, theta, out, precision="fp64"):
        code = self.lib.tnt_heff2_apply(self.ctx, L.ref, W1.ref, W2.ref, R.ref, theta.ref,
                                        out.ref, PRECISIONS[precision])
        return self._check("tnt_heff2_apply", code)

    def heff2_apply_noalloc(self, L, W1, W2, R, theta, out, precision="fp64"):
        """tnt_heff2_apply through the allocation-free entry point (blocks)."""
        code = self.lib.tnt_heff2_apply_noalloc(self.ctx, L.ref, W1.ref, W2.ref, R.ref,
                                                theta.ref, out.ref, PRECISIONS[precision])
        return self._check("tnt_heff2_apply_noalloc", code)

    def heff2_flops(self, L, W1, W2, R, theta):
        parts = np.zeros(3, dtype=np.int64)
        f = self.lib.tnt_heff2_flops(L.ref, W1.ref, W2.ref, R.ref, theta.ref, _ptr(parts, I64P))
        if f < 0:
            raise TntError("tnt_heff2_flops", -1, "invalid input")
        return int(f), parts

    def lanczos_ground(self, L, W1, W2, R, theta, kmax=20, precision="fp64", beta_tol=1e-12,
                       resid_tol=-1.0):
        p = LanczosParams(kmax, PRECISIONS[precision], beta_tol, resid_tol)
        r = LanczosResult()
        code = self.lib.tnt_lanczos_ground(self.ctx, L.ref, W1.ref, W2.ref, R.ref, theta.ref,
                                           C.byref(p), C.byref(r))
        self._check("tnt_lanczos_ground", code)
        return {"E_ritz": r.E_ritz, "E": r.E_refined, "residual": r.residual,
                "steps": r.steps, "status": code}


    def auto_block_svd(self, A, tol, chi_max, abs_tol=-1.0, rel_tol=-1.0, err_tol=-1.0,
                       err_type=TNT_ERR_2NORM, renormalise=False):
        """Truncated SVD of a dense complex matrix A (host array, m x n) through
        automatic blocking; returns dict(U, B, S, chi, nblocks, eps) with U (m x chi)
        and B (chi x n) on the host, U @ B the truncated matrix."""
        import torch
        A = np.asarray(A, dtype=complex)
        m, n = A.shape
        are = torch.from_numpy(np.ascontiguousarray(A.real)).to(self.dev)
        aim = torch.from_numpy(np.ascontiguousarray(A.imag)).to(self.dev)
        ure = torch.empty((m, chi_max), dtype=torch.float64, device=self.dev)
        uim = torch.empty_like(ure)
        bre = torch.empty((chi_max, n), dtype=torch.float64, device=self.dev)
        bim = torch.empty_like(bre)
        S = np.zeros(chi_max)
        chi = C.c_int32()
        nb = C.c_int32()
        eps = C.c_double()
        tp = TruncParams(int(chi_max), err_type, abs_tol, rel_tol, err_tol, int(bool(renormalise)))

        def fp(t):
            return C.cast(C.c_void_p(t.data_ptr()), F64P)

        self._check("tnt_auto_block_svd", self.lib.tnt_auto_block_svd(
            self.ctx, fp(are), fp(aim), m, n, n, float(tol), C.byref(tp), fp(ure), fp(uim),
            chi_max, fp(bre), fp(bim), n, S.ctypes.data_as(F64P), C.byref(chi), C.byref(nb),
            C.byref(eps)))
        k = chi.value
        U = (ure.cpu().numpy() + 1j * uim.cpu().numpy())[:, :k]
        Bm = (bre.cpu().numpy() + 1j * bim.cpu().numpy())[:k]
        return {"U": U, "B": Bm, "S": S[:k], "chi": k, "nblocks": nb.value, "eps": eps.value}

    def svd_truncate(self, theta, chi_max, abs_tol=-1.0, rel_tol=-1.0, err_tol=-1.0,
                     err_type=TNT_ERR_2NORM, renormalise=True, absorb="right"):
        """Truncated SVD of a theta descriptor; returns factors as block dicts."""
        rows, cols = {}, {}
        for (qa, s1, s2), shp in zip(theta.keys, theta.shapes):
            m = qa + s1
            rows.setdefault(m, {})[(s1, qa)] = shp[0]
            cols.setdefault(m, {})[(s2, m + s2)] = shp[1]
        capA = capB = capS = 0
        for m in rows:
            R, Cc = sum(rows[m].values()), sum(cols[m].values())
            K = min(R, Cc)
            capA += R * K
            capB += K * Cc
            capS += K
        nblk = sum(len(v) for v in rows.values()) + sum(len(v) for v in cols.values()) + 8
        outs = []
        for cap in (capA, capB):
            re, im = self.planes(cap)
            qn = np.zeros(3 * nblk, np.int32)
            ext = np.zeros(3 * nblk, np.int32)
            off = np.zeros(nblk, np.int64)
            so = SiteOut(nblk, 0, _ptr(qn, I32P), _ptr(ext, I32P), _ptr(off, I64P),
                         C.cast(C.c_void_p(re.data_ptr()), F64P),
                         C.cast(C.c_void_p(im.data_ptr()), F64P), int(re.numel()))
            outs.append((so, qn, ext, off, re, im))
        S = np.zeros(max(capS, 1), np.float64)
        bq = np.zeros(nblk, np.int32)
        bd = np.zeros(nblk, np.int32)
        p = TruncParams(int(chi_max), int(err_type), float(abs_tol), float(rel_tol),
                        float(err_tol), 1 if renormalise else 0)
        r = TruncResult()
        code = self.lib.tnt_theta_svd_truncate(
            self.ctx, theta.ref, C.byref(p),
            TNT_ABSORB_RIGHT if absorb == "right" else TNT_ABSORB_LEFT, C.byref(outs[0][0]),
            C.byref(outs[1][0]), _ptr(S, F64P), len(S), _ptr(bq, I32P), _ptr(bd, I32P),
            C.byref(r))
        self._check("tnt_theta_svd_truncate", code)
        self.sync()
        facs = []
        for (so, qn, ext, off, re, im) in outs:
            rr, ii = re.cpu().numpy(), im.cpu().numpy()
            blocks = {}
            for b in range(so.nblocks):
                nr, nc = int(ext[3 * b]), int(ext[3 * b + 2])
                o = int(off[b])
                blocks[(int(qn[3 * b]), int(qn[3 * b + 1]))] = \
                    (rr[o:o + nr * nc] + 1j * ii[o:o + nr * nc]).reshape(nr, nc)
            facs.append(blocks)
        bond = {int(bq[i]): int(bd[i]) for i in range(r.nsectors)}
        lams, pos = {}, 0
        for q in sorted(bond):
            lams[q] = S[pos:pos + bond[q]].copy()
            pos += bond[q]
        return {"A": facs[0], "B": facs[1], "bond": bond, "lambdas": lams, "chi": r.chi,
                "eps": r.eps, "lambda0": r.lambda0, "norm_kept": r.norm_kept}

    # -- MPS / environments / sweep ------------------------------------------
    def mps(self, bonds, sites, d):
        """Upload a block MPS (bonds[0..L] sector dicts, sites[0..L-1] block dicts)."""
        return Mps(self, bonds, sites, d)

    @staticmethod
    def _ptr_array(ctype, objs):
        arr = (C.POINTER(ctype) * len(objs))()
        for i, o in enumerate(objs):
            arr[i] = C.pointer(o.c)
        return arr

    def heff2_apply_batched(self, Ls, W1s, W2s, Rs, thetas, outs, precision="fp64"):
        """n independent H_eff applications in one batch (lists of descriptors)."""
        n = len(thetas)
        args = [self._ptr_array(BTensor, Ls), self._ptr_array(MpoSite, W1s),
                self._ptr_array(MpoSite, W2s), self._ptr_array(BTensor, Rs),
                self._ptr_array(BTensor, thetas), self._ptr_array(BTensor, outs)]
        code = self.lib.tnt_heff2_apply_batched(self.ctx, n, *args, PRECISIONS[precision])
        return self._check("tnt_heff2_apply_batched", code)

    def lanczos_ground_batched(self, Ls, W1s, W2s, Rs, thetas, kmax=20, precision="fp64",
                               beta_tol=1e-12, resid_tol=-1.0):
        """Batched Lanczos: one result dict per instance; thetas are updated in place."""
        n = len(thetas)
        p = LanczosParams(kmax, PRECISIONS[precision], beta_tol, resid_tol)
        rs = (LanczosResult * n)()
        args = [self._ptr_array(BTensor, Ls), self._ptr_array(MpoSite, W1s),
                self._ptr_array(MpoSite, W2s), self._ptr_array(BTensor, Rs),
                self._ptr_array(BTensor, thetas)]
        code = self.lib.tnt_lanczos_ground_batched(self.ctx, n, *args, C.byref(p), rs)
        self._check("tnt_lanczos_ground_batched", code)
        return [{"E_ritz": r.E_ritz, "E": r.E_refined, "residual": r.residual, "steps": r.steps,
                 "status": code} for r in rs]

    def sweep_batched(self, mpss, envs, chi_max, kmax=20, precision="fp64", rel_tol=1e-12,
                      abs_tol=-1.0, err_tol=-1.0, err_type=TNT_ERR_2NORM, beta_tol=1e-12):
        """One lockstep sweep of several chains; chi_max per chain (list) or common."""
        n = len(mpss)
        chis = list(chi_max) if hasattr(chi_max, "__len__") else [chi_max] * n
        ps = (SweepParams * n)()
        rec = []
        for i, m in enumerate(mpss):
            cap = 2 * (m.L - 1)
            arr = (np.zeros(cap), np.zeros(cap), np.zeros(cap, np.int32), np.zeros(cap, np.int32))
            rec.append(arr)
            ps[i] = SweepParams(LanczosParams(kmax, PRECISIONS[precision], beta_tol, -1.0),
                                TruncParams(int(chis[i]), int(err_type), float(abs_tol),
                                            float(rel_tol), float(err_tol), 1),
                                cap, _ptr(arr[0], F64P), _ptr(arr[1], F64P), _ptr(arr[2], I32P),
                                _ptr(arr[3], I32P))
        hm = (P * n)(*[m.h.value for m in mpss])
        he = (P * n)(*[e.h.value for e in envs])
        rs = (SweepResult * n)()
        code = self.lib.tnt_dmrg_sweep_batched(self.ctx, n, hm, he, ps, rs)
        self._check("tnt_dmrg_sweep_batched", code)
        out = []
        for r, (E, eps, chi, steps) in zip(rs, rec):
            d = {f: getattr(r, f) for f, _ in SweepResult._fields_}
            d.update({"bond_E": E, "bond_eps": eps, "bond_chi": chi, "bond_steps": steps})
            out.append(d)
        return out

    def tebd_step(self, mps, h, dt, chi_max, rel_tol=1e-12, abs_tol=-1.0, err_tol=-1.0,
                  err_type=TNT_ERR_2NORM, renormalise=True):
        """One second-order TEBD step of dt with bond Hamiltonians h
        (L-1, d^2, d^2); returns per-gate truncation errors, kept dims, stats.
        The default relative cut (as in sweep) drops Schmidt values below
        1e-12 of the largest; rel_tol=-1 keeps up to chi_max values."""
        h = np.ascontiguousarray(h, dtype=np.float64)
        cap = 2 * (mps.L - 1)
        eps = np.zeros(cap)
        chi = np.zeros(cap, np.int32)
        stats = np.zeros(6)
        tp = TruncParams(int(chi_max), err_type, abs_tol, rel_tol, err_tol, int(bool(renormalise)))
        self._check("tnt_tebd_step", self.lib.tnt_tebd_step(
            self.ctx, mps.h, h.ctypes.data_as(F64P), float(dt), C.byref(tp), cap,
            eps.ctypes.data_as(F64P), chi.ctypes.data_as(I32P), stats.ctypes.data_as(F64P)))
        return {"bond_eps": eps.tolist(), "bond_chi": chi.tolist(), "seconds_total": stats[0],
                "seconds_gate": stats[1], "seconds_svd": stats[2], "sum_eps": stats[3],
                "max_eps": stats[4], "max_chi": int(stats[5])}

    def bond_hamiltonians_bose_hubbard(self, L, nmax, J, U, mu=0.0):
        return bond_hamiltonians_bose_hubbard(self.lib, L, nmax, J, U, mu)

    def bond_hamiltonians_spin1(self, L, J=1.0):
        return bond_hamiltonians_spin1(self.lib, L, J)

    def sweep(self, mps, env, chi_max, kmax=20, precision="fp64", rel_tol=1e-12, abs_tol=-1.0,
              err_tol=-1.0, err_type=TNT_ERR_2NORM, beta_tol=1e-12):
        L = mps.L
        cap = 2 * (L - 1)
        E = np.zeros(cap)
        eps = np.zeros(cap)
        chi = np.zeros(cap, np.int32)
        steps = np.zeros(cap, np.int32)
        p = SweepParams(LanczosParams(kmax, PRECISIONS[precision], beta_tol, -1.0),
                        TruncParams(int(chi_max), int(err_type), float(abs_tol), float(rel_tol),
                                    float(err_tol), 1),
                        cap, _ptr(E, F64P), _ptr(eps, F64P), _ptr(chi, I32P), _ptr(steps, I32P))
        r = SweepResult()
        code = self.lib.tnt_dmrg_sweep(self.ctx, mps.h, env.h, C.byref(p), C.byref(r))
        self._check("tnt_dmrg_sweep", code)
        out = {f: getattr(r, f) for f, _ in SweepResult._fields_}
        out.update({"bond_E": E, "bond_eps": eps, "bond_chi": chi, "bond_steps": steps})
        return out


class Mps:
    """Device MPS handle (tnt_mps)."""

    def __init__(self, tnt: Tnt, bonds, sites, d):
        self.t = tnt
        self.L = len(sites)
        self.d = int(d)
        h = P()
        tnt._check("tnt_mps_create", tnt.lib.tnt_mps_create(tnt.ctx, self.L, self.d, C.byref(h)))
        self.h = h
        for ell, b in enumerate(bonds):
            q = _i32(sorted(b))
            dm = _i32([b[k] for k in sorted(b)])
            tnt._check("tnt_mps_set_bond",
                       tnt.lib.tnt_mps_set_bond(h, ell, len(q), _ptr(q, I32P), _ptr(dm, I32P)))
        for j, site in enumerate(sites, start=1):
            keys = sorted(site)
            ql = _i32([k[0] for k in keys])
            ss = _i32([k[1] for k in keys])
            flat = np.concatenate([site[k].reshape(-1) for k in keys]) if keys else \
                np.zeros(0, complex)
            re = np.ascontiguousarray(flat.real)
            im = np.ascontiguousarray(flat.imag)
            tnt._check("tnt_mps_set_site",
                       tnt.lib.tnt_mps_set_site(h, j, len(keys), _ptr(ql, I32P), _ptr(ss, I32P),
                                                _ptr(re, F64P), _ptr(im, F64P)))

    def __del__(self):
        try:
            if self.h:
                self.t.lib.tnt_mps_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def right_canonicalize(self):
        self.t._check("tnt_mps_right_canonicalize",
                      self.t.lib.tnt_mps_right_canonicalize(self.t.ctx, self.h))

    def correlation(self, op, dq, with_flops=False):
        """C[i, j] = <O^dagger_i O_j> (0-based) for a real operator matrix
        op[s', s] = <s'|O|s> that changes the charge by dq."""
        op = np.ascontiguousarray(op, dtype=np.float64)
        L = self.L
        re = np.zeros((L, L))
        im = np.zeros((L, L))
        fl = C.c_double()
        self.t._check("tnt_mps_correlation", self.t.lib.tnt_mps_correlation(
            self.t.ctx, self.h, op.ctypes.data_as(F64P), int(dq), re.ctypes.data_as(F64P),
            im.ctypes.data_as(F64P), C.byref(fl)))
        out = re + 1j * im
        return (out, fl.value) if with_flops else out

    def bond(self, ell):
        n = self.t.lib.tnt_mps_bond_size(self.h, ell)
        q = np.zeros(max(n, 1), np.int32)
        dm = np.zeros(max(n, 1), np.int32)
        self.t._check("tnt_mps_get_bond",
                      self.t.lib.tnt_mps_get_bond(self.h, ell, n, _ptr(q, I32P), _ptr(dm, I32P)))
        return {int(q[i]): int(dm[i]) for i in range(n)}

    def bonds(self):
        return [self.bond(ell) for ell in range(self.L + 1)]

    def site(self, j):
        left, right = self.bond(j - 1), self.bond(j)
        cap = len(left) * self.d + 1
        ecap = sum(left.values()) * sum(right.values()) * self.d + 1
        ql = np.zeros(cap, np.int32)
        ss = np.zeros(cap, np.int32)
        re = np.zeros(ecap)
        im = np.zeros(ecap)
        nb = C.c_int32()
        self.t._check("tnt_mps_get_site",
                      self.t.lib.tnt_mps_get_site(self.h, j, cap, C.byref(nb), _ptr(ql, I32P),
                                                  _ptr(ss, I32P), ecap, _ptr(re, F64P),
                                                  _ptr(im, F64P)))
        out, pos = {}, 0
        for i in range(nb.value):
            q, s = int(ql[i]), int(ss[i])
            r, c = left[q], right[q + s]
            out[(q, s)] = (re[pos:pos + r * c] + 1j * im[pos:pos + r * c]).reshape(r, c)
            pos += r * c
        return out

    def sites(self):
        return [self.site(j) for j in range(1, self.L + 1)]


class Env:
    """Device environment handle (tnt_env) for an MPS and a chain MPO."""

    def __init__(self, tnt: Tnt, mps: Mps, W_list, qw, left_index=3, right_index=0):
        self.t = tnt
        self.mpos = [Mpo(W, qw) for W in W_list]
        arr = (MpoSite * len(self.mpos))(*[m.c for m in self.mpos])
        self._arr = arr
        h = P()
        tnt._check("tnt_env_create", tnt.lib.tnt_env_create(tnt.ctx, mps.h, arr, left_index,
                                                            right_index, C.byref(h)))
        self.h = h

    def __del__(self):
        try:
            if self.h:
                self.t.lib.tnt_env_destroy(self.h)
                self.h = None
        except Exception:
            pass


_SINGLETON = None


def load() -> Tnt:
    """The process-wide context on cuda:0 (created on first use)."""
    global _SINGLETON
    if _SINGLETON is None:
        _SINGLETON = Tnt(0)
    return _SINGLETON
