"""ctypes binding of libcamg (the C-ABI declared in include/camg.h).

Argument marshalling only: every step of the solve runs inside the HIP
library.  Function names match the C entry points; `AMGSolver` bundles a
handle with torch-allocated device vectors for convenience.

PyTorch supplies device memory and streams.  torch is imported before the
library is loaded so that both share one HIP runtime in the process.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, byref, c_char_p, c_double, c_int, c_int32, c_int64, c_void_p
from dataclasses import dataclass

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcamg.so")

CAMG_OK = 0
CAMG_NOT_CONVERGED = 1
PREC_FP64 = 0
PREC_MIXED = 1
PREC_MIXED_BF16 = 2
SPMV_AUTO, SPMV_CSR, SPMV_BELL, SPMV_FULL = 0, 1, 2, 4
KCLASS_SMOOTH_U = 1
KCLASS_OPERATOR = 2
KCLASS_ORTHO = 4
KCLASS_RESIDUAL = 8


class amg_csr(Structure):
    _fields_ = [
        ("nrows", c_int64),
        ("ncols", c_int64),
        ("nnz", c_int64),
        ("rowptr", POINTER(c_int64)),
        ("col", POINTER(c_int32)),
        ("val", POINTER(c_double)),
    ]


class amg_problem(Structure):
    _fields_ = [
        ("dim", c_int32),
        ("K", amg_csr),
        ("G", amg_csr),
        ("B", amg_csr),
        ("C", amg_csr),
        ("n_slave", c_int32),
        ("n_master", c_int32),
        ("slave_dofs", POINTER(c_int32)),
        ("master_dofs", POINTER(c_int32)),
        ("lm_node", POINTER(c_int32)),
        ("n_ns", c_int32),
        ("nullspace", POINTER(c_double)),
        ("device_ptrs", c_int32),
    ]


class amg_options(Structure):
    _fields_ = [
        ("max_levels", c_int32),
        ("max_coarse_rows", c_int32),
        ("nu_pre", c_int32),
        ("nu_post", c_int32),
        ("jacobi_sweeps", c_int32),
        ("atilde", c_int32),
        ("jacobi_diag", c_int32),
        ("precision", c_int32),
        ("spmv_format", c_int32),
        ("graphs", c_int32),
        ("jacobi_omega", c_double),
        ("simple_alpha", c_double),
        ("prolongator", c_int32),
        ("schur", c_int32),
        ("schur_sweeps", c_int32),
        ("sa_omega", c_double),
        ("coarse_solver", c_int32),
        ("coarse_sweeps", c_int32),
        ("smoother", c_int32),
    ]


class amg_gmres_options(Structure):
    _fields_ = [
        ("m", c_int32),
        ("max_iters", c_int32),
        ("fixed_iters", c_int32),
        ("lookahead", c_int32),
        ("rtol", c_double),
        ("ortho", c_int32),
    ]


class amg_gmres_result(Structure):
    _fields_ = [
        ("iters", c_int32),
        ("restarts", c_int32),
        ("status", c_int32),
        ("rel_res_est", c_double),
        ("rel_res_true", c_double),
        ("seconds", c_double),
    ]


class amg_level_info(Structure):
    _fields_ = [
        ("n_u", c_int64),
        ("n_l", c_int64),
        ("nnz_K", c_int64),
        ("nnz_G", c_int64),
        ("nnz_B", c_int64),
        ("nnz_C", c_int64),
        ("bs_u", c_int32),
        ("bs_l", c_int32),
        ("n_nodes_u", c_int64),
        ("n_nodes_l", c_int64),
        ("n_agg_u", c_int64),
        ("n_agg_l", c_int64),
        ("op_complexity", c_double),
        ("k_layout", c_int32),
        ("k_bs", c_int32),
        ("k_blocks", c_int64),
        ("k_slots", c_int64),
        ("transfer_layout", c_int32),
        ("k_index_bytes", c_int32),
        ("k_lower_blocks", c_int64),
        ("k_nnz_stored", c_int64),
        ("k_sym_stale", c_int32),
    ]


# name -> (restype, argtypes); every symbol declared in include/camg.h
SIGNATURES = {
    "amg_default_options": (None, [POINTER(amg_options)]),
    "amg_default_gmres_options": (None, [POINTER(amg_gmres_options)]),
    "amg_setup": (c_int, [POINTER(amg_problem), POINTER(amg_options), c_void_p, POINTER(c_void_p)]),
    "amg_setup_host": (c_int, [POINTER(amg_problem), POINTER(amg_options), POINTER(c_void_p)]),
    "amg_num_levels": (c_int, [c_void_p]),
    "amg_level_info_get": (c_int, [c_void_p, c_int, POINTER(amg_level_info)]),
    "amg_get_aggregates": (c_int, [c_void_p, c_int, POINTER(c_int32), POINTER(c_int32)]),
    "amg_get_level_matrix": (
        c_int,
        [c_void_p, c_int, c_int, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64), POINTER(c_int64),
         POINTER(c_int32), POINTER(c_double)],
    ),
    "amg_update_fine_values": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "amg_apply_operator": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "amg_vcycle_apply": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "amg_vcycle_apply_noalloc": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "fgmres_solve": (
        c_int,
        [c_void_p, c_int, c_void_p, c_void_p, POINTER(amg_gmres_options), POINTER(amg_gmres_result), c_void_p],
    ),
    "amg_grad_K": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "amg_grad_A": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "amg_dense_inverse": (c_int, [c_void_p, c_void_p, c_int64, c_void_p]),
    "amg_profile_enable": (c_int, [c_void_p, c_int]),
    "amg_profile_read": (c_int, [c_void_p, c_int, POINTER(c_int64), POINTER(c_double)]),
    "amg_destroy": (None, [c_void_p]),
    "amg_strerror": (c_char_p, [c_int]),
    "amg_last_error": (c_char_p, []),
}

_lib = None


def load_library(path: str = _LIB_PATH):
    """Load libcamg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libcamg.so not found at {path}: build the HIP library first "
            "(python -m paper_1912_09056_amd.build)"
        )
    lib = ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class CamgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libcamg error {code}: {msg}")
        self.code = code


def _check(code):
    if code < 0:
        lib = load_library()
        raise CamgError(code, f"{lib.amg_strerror(code).decode()} ({lib.amg_last_error().decode()})")
    return code


@dataclass
class AMGOptions:
    max_levels: int = 4
    max_coarse_rows: int = 1000
    nu_pre: int = 2
    nu_post: int = 2
    jacobi_sweeps: int = 1
    atilde: int = 0  # SIMPLEC lumping: 0 row sums of |K|, 1 diag(K), 2 nodal blocks (rotation-covariant)
    jacobi_diag: int = 0
    precision: int = PREC_FP64
    # 0 auto, 1 CSR, 2 sliced blocked-ELL; | 4 (SPMV_FULL): a K equal to its
    # transpose stays in full blocked-ELL instead of symmetric storage
    spmv_format: int = 0
    graphs: int = 1  # replay the V-cycle from a captured HIP graph
    jacobi_omega: float = 0.8
    simple_alpha: float = 0.8
    prolongator: int = 0  # 0 tentative, 1 smoothed aggregation (displacement transfers)
    schur: int = 0  # Schur relaxation: 0 diag(S), 1 signed l1 row sums, 2 nodal diagonal blocks of S
    schur_sweeps: int = 1  # (block) Jacobi sweeps on the Schur system (1 = division by the diagonal / blocks)
    sa_omega: float = 4.0 / 3.0
    coarse_solver: int = 0  # coarsest level: 0 dense LU inverse, 1 CheapSIMPLE sweeps
    coarse_sweeps: int = 2
    smoother: int = 0  # 0 CheapSIMPLE, 1 inexact Uzawa, 2 cheap Braess-Sarazin (simple_alpha is the block damping)

    @classmethod
    def robust(cls, **overrides) -> "AMGOptions":
        """Settings for strong stiffness contrast, after the paper's
        weak-scaling configuration: smoothed aggregation (omega 4/3), three
        CheapSIMPLE sweeps per level with a two-sweep prediction, and eight
        l1-lumped Jacobi sweeps on the Schur system in place of its ILU.  The
        default settings stall on lognormal(0, 2) moduli at 150^3."""
        kw = dict(prolongator=1, schur=1, schur_sweeps=8, jacobi_sweeps=2, nu_pre=3, nu_post=3)
        kw.update(overrides)
        return cls(**kw)

    @classmethod
    def rotation_robust(cls, **overrides) -> "AMGOptions":
        """Nodal lumping and nodal Schur blocks: every smoother covariant
        under rigid rotations of the geometry (interfaces whose normals are
        not coordinate axes)."""
        kw = dict(atilde=2, schur=2)
        kw.update(overrides)
        return cls(**kw)

    def to_c(self) -> amg_options:
        o = amg_options()
        for f in amg_options._fields_:
            setattr(o, f[0], getattr(self, f[0]))
        return o


def _ptr(a, ctype):
    return a.ctypes.data_as(POINTER(ctype)) if a is not None and a.size else None


def _csr_arrays(M, nrows, ncols):
    """(rowptr int64, col int32, val float64, shape) from a scipy-like CSR
    matrix; None is an empty nrows x ncols block.  The shape is passed on as
    the matrix has it: the library checks it against the system."""
    if M is None:
        return np.zeros(nrows + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float64), (nrows, ncols)
    M = M.tocsr()
    M.sort_indices()
    return (
        np.ascontiguousarray(M.indptr, dtype=np.int64),
        np.ascontiguousarray(M.indices, dtype=np.int32),
        np.ascontiguousarray(M.data, dtype=np.float64),
        M.shape,
    )


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def _dptr(t: torch.Tensor):
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
    return c_void_p(t.data_ptr())


class AMGSolver:
    """Owns one libcamg handle built from a contact problem.

    K, G, B, C: scipy CSR matrices (host); slave_dofs / master_dofs: int
    arrays of interface displacement dofs; nullspace: (n_u, n_ns) array.
    """

    def __init__(self, dim, K, G, B, C, slave_dofs, master_dofs, nullspace=None, lm_node=None,
                 options: AMGOptions = None, device=None, host_only: bool = False):
        n_u, n_l = K.shape[0], C.shape[0]
        keep = []
        prob = amg_problem()
        prob.dim = dim
        for name, M, r, c in (("K", K, n_u, n_u), ("G", G, n_u, n_l), ("B", B, n_l, n_u), ("C", C, n_l, n_l)):
            rp, ci, v, (mr, mc) = _csr_arrays(M, r, c)
            keep += [rp, ci, v]
            setattr(prob, name, amg_csr(mr, mc, ci.size, _ptr(rp, c_int64), _ptr(ci, c_int32), _ptr(v, c_double)))
        sd = np.ascontiguousarray(slave_dofs, dtype=np.int32)
        md = np.ascontiguousarray(master_dofs, dtype=np.int32)
        keep += [sd, md]
        prob.n_slave, prob.n_master = sd.size, md.size
        prob.slave_dofs, prob.master_dofs = _ptr(sd, c_int32), _ptr(md, c_int32)
        if lm_node is not None:
            ln = np.ascontiguousarray(lm_node, dtype=np.int32)
            keep.append(ln)
            prob.lm_node = _ptr(ln, c_int32)
        if nullspace is not None:
            ns = np.asfortranarray(nullspace, dtype=np.float64)
            flat = np.ascontiguousarray(ns.reshape(-1, order="F"))
            keep.append(flat)
            prob.n_ns = ns.shape[1]
            prob.nullspace = _ptr(flat, c_double)
        nnz = {"K": keep[2].size, "G": keep[5].size, "B": keep[8].size, "C": keep[11].size}
        self._finish(prob, n_u, n_l, dim, nnz, options, device, host_only)

    def _finish(self, prob, n_u, n_l, dim, nnz, options, device, host_only):
        self.lib = load_library()
        self.host_only = host_only
        if host_only:
            self.device = None
        else:
            self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.options = options or AMGOptions()
        self.n_u, self.n_l, self.n = n_u, n_l, n_u + n_l
        self.dim = dim
        self.K_nnz = nnz["K"]
        self.block_nnz = dict(nnz)
        h = c_void_p()
        opts = self.options.to_c()
        if host_only:
            _check(self.lib.amg_setup_host(byref(prob), byref(opts), byref(h)))
        else:
            with torch.cuda.device(self.device):
                _check(self.lib.amg_setup(byref(prob), byref(opts), _stream_ptr(), byref(h)))
        self.handle = h
        self.n_levels = self.lib.amg_num_levels(h)

    @classmethod
    def from_device(cls, dim, blocks, slave_dofs, master_dofs, nullspace=None, lm_node=None,
                    options: AMGOptions = None):
        """Setup from device-resident arrays (device_ptrs = 1): `blocks` maps
        "K", "G", "B", "C" to (rowptr int64, col int32, val float64, (nrows,
        ncols)) with the arrays as CUDA tensors on the current device;
        slave_dofs / master_dofs / lm_node int32 and nullspace float64
        (n_u x n_ns, column-major: a tensor of shape (n_ns, n_u)) likewise.
        The library copies them down to build the hierarchy."""
        self = cls.__new__(cls)
        dev = torch.device("cuda", torch.cuda.current_device())

        def dp(t, dtype, ctype):
            if t is None or t.numel() == 0:
                return None, None
            t = t.to(device=dev, dtype=dtype).contiguous()
            return t, ctypes.cast(c_void_p(t.data_ptr()), POINTER(ctype))

        keep = []
        prob = amg_problem()
        prob.dim = dim
        nnz = {}
        for name in ("K", "G", "B", "C"):
            rp, ci, v, (nr, nc) = blocks[name]
            trp, prp = dp(rp, torch.int64, c_int64)
            tci, pci = dp(ci, torch.int32, c_int32)
            tv, pv = dp(v, torch.float64, c_double)
            keep += [trp, tci, tv]
            nnz[name] = 0 if tci is None else tci.numel()
            setattr(prob, name, amg_csr(nr, nc, nnz[name], prp, pci, pv))
        tsd, psd = dp(torch.as_tensor(slave_dofs), torch.int32, c_int32)
        tmd, pmd = dp(torch.as_tensor(master_dofs), torch.int32, c_int32)
        keep += [tsd, tmd]
        prob.n_slave = 0 if tsd is None else tsd.numel()
        prob.n_master = 0 if tmd is None else tmd.numel()
        prob.slave_dofs, prob.master_dofs = psd, pmd
        if lm_node is not None:
            tln, prob.lm_node = dp(torch.as_tensor(lm_node), torch.int32, c_int32)
            keep.append(tln)
        if nullspace is not None:
            tns, prob.nullspace = dp(torch.as_tensor(nullspace), torch.float64, c_double)
            keep.append(tns)
            prob.n_ns = tns.shape[0]
        prob.device_ptrs = 1
        torch.cuda.synchronize()
        n_u, n_l = blocks["K"][3][0], blocks["C"][3][0]
        self._finish(prob, n_u, n_l, dim, nnz, options, dev.index, False)
        return self

    def __del__(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            try:
                self.lib.amg_destroy(self.handle)
            except Exception:
                pass
            self.handle = None

    @classmethod
    def from_problem(cls, prob, options: AMGOptions = None, device=None, host_only: bool = False):
        return cls(prob.dim, prob.K, prob.G, prob.B, prob.C, prob.slave_dofs, prob.master_dofs,
                   nullspace=prob.nullspace, lm_node=prob.lm_node, options=options, device=device,
                   host_only=host_only)

    # ---- queries ---------------------------------------------------------
    def level_info(self, level: int) -> dict:
        info = amg_level_info()
        _check(self.lib.amg_level_info_get(self.handle, level, byref(info)))
        return {f[0]: getattr(info, f[0]) for f in amg_level_info._fields_}

    def aggregates(self, level: int):
        info = self.level_info(level)
        du = np.zeros(info["n_nodes_u"], np.int32)
        dl = np.zeros(info["n_nodes_l"], np.int32)
        _check(self.lib.amg_get_aggregates(self.handle, level, _ptr(du, c_int32), _ptr(dl, c_int32)))
        return du, dl

    def level_matrix(self, level: int, which: str):
        """Host copy of block K/G/B/C/P_u/P_l/S/Sblk_inv/Ablk_inv of a level as
        scipy CSR (S: the Schur matrix, kept only with schur_sweeps > 1;
        Sblk_inv: the inverse nodal blocks of S with the block Schur option;
        Ablk_inv: the inverse nodal lumping blocks with atilde=2; else
        0 x 0)."""
        import scipy.sparse as sp

        w = {"K": 0, "G": 1, "B": 2, "C": 3, "P_u": 4, "P_l": 5, "S": 6, "Sblk_inv": 7, "Ablk_inv": 8}[which]
        nr, nc, nz = c_int64(), c_int64(), c_int64()
        _check(self.lib.amg_get_level_matrix(self.handle, level, w, byref(nr), byref(nc), byref(nz), None, None, None))
        rp = np.zeros(nr.value + 1, np.int64)
        ci = np.zeros(nz.value, np.int32)
        v = np.zeros(nz.value, np.float64)
        _check(self.lib.amg_get_level_matrix(self.handle, level, w, None, None, None, _ptr(rp, c_int64),
                                             _ptr(ci, c_int32), _ptr(v, c_double)))
        return sp.csr_matrix((v, ci, rp), shape=(nr.value, nc.value))

    # ---- device work -------------------------------------------------------
    def _vec(self, x):
        if x is None:
            return torch.zeros(self.n, dtype=torch.float64, device=self.device)
        t = torch.as_tensor(x, dtype=torch.float64, device=self.device)
        return t.contiguous()

    def apply_operator(self, x, transpose=False, stream=None):
        x = self._vec(x)
        y = torch.empty_like(x)
        _check(self.lib.amg_apply_operator(self.handle, int(transpose), _dptr(x), _dptr(y), _stream_ptr(stream)))
        return y

    def vcycle(self, r, transpose=False, stream=None):
        r = self._vec(r)
        z = torch.empty_like(r)
        _check(self.lib.amg_vcycle_apply(self.handle, int(transpose), _dptr(r), _dptr(z), _stream_ptr(stream)))
        return z

    def vcycle_noalloc(self, r, z, transpose=False, stream=None):
        """z = M^-1 r (or M^-T r) through the allocation-free entry point;
        r and z are caller-owned FP64 device vectors of length n."""
        _check(self.lib.amg_vcycle_apply_noalloc(self.handle, int(transpose), _dptr(r), _dptr(z),
                                                 _stream_ptr(stream)))
        return z

    def solve(self, b, x0=None, transpose=False, m=50, rtol=1e-8, max_iters=1000, fixed_iters=0, lookahead=1,
              stream=None, ortho=1):
        """FGMRES solve; returns (x, result dict).  ortho: 1 two-pass CGS2
        (Gram-matrix second projection), 0 three-pass CGS2."""
        b = self._vec(b)
        x = self._vec(x0).clone() if x0 is not None else torch.zeros_like(b)
        go = amg_gmres_options(m, max_iters, fixed_iters, lookahead, rtol, ortho)
        res = amg_gmres_result()
        code = _check(self.lib.fgmres_solve(self.handle, int(transpose), _dptr(b), _dptr(x), byref(go), byref(res),
                                            _stream_ptr(stream)))
        out = {f[0]: getattr(res, f[0]) for f in amg_gmres_result._fields_}
        out["converged"] = code == CAMG_OK
        return x, out

    def grad_K(self, lam, x, stream=None):
        lam, x = self._vec(lam), self._vec(x)
        dK = torch.empty(self.K_nnz, dtype=torch.float64, device=self.device)
        _check(self.lib.amg_grad_K(self.handle, _dptr(lam), _dptr(x), _dptr(dK), _stream_ptr(stream)))
        return dK

    def grad_A(self, lam, x, blocks=("K", "G", "B", "C"), stream=None):
        """{block: -lam_i x_j on that block's stored entries} for the named
        blocks of A = [[K, G], [B, C]]."""
        lam, x = self._vec(lam), self._vec(x)
        out = {name: torch.empty(self.block_nnz[name], dtype=torch.float64, device=self.device) for name in blocks}
        args = [_dptr(out[name]) if name in out else None for name in ("K", "G", "B", "C")]
        _check(self.lib.amg_grad_A(self.handle, _dptr(lam), _dptr(x), *args, _stream_ptr(stream)))
        return out

    def update_fine_values(self, K_val=None, G_val=None, B_val=None, C_val=None, stream=None):
        args = []
        keep = []
        for v in (K_val, G_val, B_val, C_val):
            if v is None:
                args.append(None)
            else:
                t = torch.as_tensor(v, dtype=torch.float64, device=self.device).contiguous()
                keep.append(t)
                args.append(_dptr(t))
        _check(self.lib.amg_update_fine_values(self.handle, *args, _stream_ptr(stream)))
        # the copies read the temporaries in `keep` asynchronously on that stream
        (stream if stream is not None else torch.cuda.current_stream(self.device)).synchronize()

    def profile_enable(self, mask: int):
        _check(self.lib.amg_profile_enable(self.handle, mask))

    def profile_read(self, kclass: int):
        n, ms = c_int64(), c_double()
        _check(self.lib.amg_profile_read(self.handle, kclass, byref(n), byref(ms)))
        return n.value, ms.value


def dense_inverse(A: torch.Tensor, stream=None) -> torch.Tensor:
    """A^-1 of a dense square FP64 CUDA matrix by the library's device LU
    (amg_dense_inverse)."""
    lib = load_library()
    A = A.to(dtype=torch.float64).contiguous()
    assert A.is_cuda and A.dim() == 2 and A.shape[0] == A.shape[1]
    out = torch.empty_like(A)
    _check(lib.amg_dense_inverse(_dptr(A), _dptr(out), A.shape[0], _stream_ptr(stream)))
    return out


def exported_symbols():
    return list(SIGNATURES)
