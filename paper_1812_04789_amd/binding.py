"""Thin ctypes binding of the C ABI in include/dg.h.

Argument marshalling only: every step of the method runs in the HIP library
libdg_mi355x.so.  PyTorch provides device memory (float64 CUDA tensors) and the
HIP stream.  Importing this module does not need a GPU; creating a Context does,
and fails loudly if the library is not built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdg_mi355x.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EHIP, DG_ENOCONV, DG_ENONFINITE, DG_ESTATE = 0, -1, -2, -3, -4, -5, -6
DG_FP64, DG_FP32, DG_BF16 = 0, 1, 2
KERNEL_KINDS = ["residual", "jvp_fd", "jvp_exact", "diag_blocks", "lu", "bj_fine", "bsr", "bj_coarse", "arnoldi"]
STATUS = {0: "DG_OK", -1: "DG_EINVAL", -2: "DG_ENOMEM", -3: "DG_EHIP", -4: "DG_ENOCONV",
          -5: "DG_ENONFINITE", -6: "DG_ESTATE"}


class MeshDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("vtx", ctypes.POINTER(ctypes.c_double))]


class Phys(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("Pr", ctypes.c_double),
                ("eta", ctypes.c_double)]


class PmgOpts(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("p_level", ctypes.c_int * 4), ("nu_pre", ctypes.c_int),
                ("nu_post", ctypes.c_int), ("omega", ctypes.c_double), ("coarsest_iters", ctypes.c_int),
                ("prec_fine", ctypes.c_int), ("prec_coarse", ctypes.c_int), ("coarse_matrix_free", ctypes.c_int),
                ("coarsest_plain", ctypes.c_int), ("smoother", ctypes.c_int), ("cycle", ctypes.c_int),
                ("coarsest_prec", ctypes.c_int)]


class FgmresOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("max_restarts", ctypes.c_int), ("rtol", ctypes.c_double),
                ("jvp_exact", ctypes.c_int)]


class FgmresStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("rel_res_true", ctypes.c_double),
                ("rel_res_est", ctypes.c_double)]


class StepStats(ctypes.Structure):
    _fields_ = [("newton", ctypes.c_int), ("linear_iters", ctypes.c_int), ("res0", ctypes.c_double),
                ("res_final", ctypes.c_double), ("max_rel_res_true", ctypes.c_double),
                ("setup_seconds", ctypes.c_double), ("solve_seconds", ctypes.c_double)]


class CaseDesc(ctypes.Structure):
    _fields_ = [("mesh", MeshDesc), ("phys", Phys), ("p", ctypes.c_int)]


class BatchTile(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int), ("epb", ctypes.c_int * 5), ("grid", ctypes.c_int),
                ("lds_bytes", ctypes.c_size_t), ("ms", ctypes.c_double), ("candidates", ctypes.c_int),
                ("items", ctypes.c_int)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int), ("hbm_budget", ctypes.c_double), ("cache", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("mesh", MeshDesc), ("phys", Phys), ("p", ctypes.c_int), ("dt", ctypes.c_double),
                ("popts", PmgOpts), ("fopts", FgmresOpts), ("newton_rtol", ctypes.c_double),
                ("max_newton", ctypes.c_int), ("Wn", ctypes.c_void_p), ("Wnm1", ctypes.c_void_p),
                ("Wnp1", ctypes.c_void_p), ("tag", ctypes.c_longlong)]


class Response(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_longlong), ("status", ctypes.c_int), ("concurrent", ctypes.c_int),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("footprint", ctypes.c_double), ("device_bytes", ctypes.c_double), ("ndof", ctypes.c_size_t),
                ("stats", StepStats)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_longlong), ("completed", ctypes.c_longlong), ("pending", ctypes.c_longlong),
                ("running", ctypes.c_int), ("contexts", ctypes.c_int), ("held_bytes", ctypes.c_double),
                ("peak_held_bytes", ctypes.c_double), ("budget_bytes", ctypes.c_double)]


# name -> (restype, argtypes)
_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
SIGNATURES = {
    "dg_create": (_I, [ctypes.POINTER(MeshDesc), ctypes.POINTER(Phys), _I, _P, ctypes.POINTER(_P)]),
    "dg_destroy": (_I, [_P]),
    "dg_ndof": (ctypes.c_size_t, [_P]),
    "dg_last_error": (ctypes.c_char_p, [_P]),
    "dg_quad_points": (_I, [_P, _P]),
    "dg_project": (_I, [_P, _P, _P]),
    "dg_residual": (_I, [_P, _P, _P]),
    "dg_jvp": (_I, [_P, _P, _P, _P, _D, _P]),
    "dg_jvp_exact": (_I, [_P, _P, _P, _D, _P]),
    "dg_mass": (_I, [_P, _P, _P]),
    "dg_assemble_diag": (_I, [_P, _P, _D, _P]),
    "dg_assemble_diag_noalloc": (_I, [_P, _P, _D, _P]),
    "dg_assemble_coarse": (_I, [_P, _P, _I, _P]),
    "dg_assemble_operator": (_I, [_P, _P, _D]),
    "dg_jvp_assembled": (_I, [_P, _P, _P]),
    "dg_batched_lu": (_I, [_P, _P, _P, _I, _I]),
    "dg_batched_lu_solve": (_I, [_P, _P, _P, _P, _P, _I, _I]),
    "pmg_setup": (_I, [_P, _P, _D, ctypes.POINTER(PmgOpts)]),
    "pmg_apply": (_I, [_P, _P, _P]),
    "fgmres_step": (_I, [_P, _P, _P, _P, _P, ctypes.POINTER(FgmresOpts), ctypes.POINTER(FgmresStats)]),
    "dg_use_graphs": (_I, [_P, _I]),
    "dg_timing": (_I, [_P, _I]),
    "dg_timing_read": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_I), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "dg_bdf2_step": (_I, [_P, _P, _P, _D, ctypes.POINTER(PmgOpts), ctypes.POINTER(FgmresOpts), _D, _I, _P,
                          ctypes.POINTER(StepStats)]),
    "dg_esdirk3_step": (_I, [_P, _P, _D, ctypes.POINTER(PmgOpts), ctypes.POINTER(FgmresOpts), _D, _I, _P,
                             ctypes.POINTER(StepStats)]),
    "dg_batch_create": (_I, [ctypes.POINTER(CaseDesc), _I, _P, ctypes.POINTER(_P)]),
    "dg_batch_destroy": (_I, [_P]),
    "dg_batch_last_error": (ctypes.c_char_p, [_P]),
    "dg_batch_ndof": (ctypes.c_size_t, [_P, _I]),
    "dg_batch_offset": (ctypes.c_size_t, [_P, _I]),
    "dg_batch_case": (_P, [_P, _I]),
    "dg_batch_residual": (_I, [_P, _P, _P]),
    "dg_batch_jvp": (_I, [_P, _P, _P, _P, _D, _P]),
    "dg_batch_jvp_exact": (_I, [_P, _P, _P, _D, _P]),
    "dg_batch_use_graphs": (_I, [_P, _I]),
    "dg_batch_get_tile": (_I, [_P, _I, ctypes.POINTER(BatchTile)]),
    "dg_batch_set_tile": (_I, [_P, _I, _I, ctypes.c_size_t, _I]),
    "dg_batch_tune": (_I, [_P, _I, _P, _P, _P, _I, ctypes.POINTER(BatchTile)]),
    "dg_batch_bdf2_step": (_I, [_P, _P, _P, _D, ctypes.POINTER(PmgOpts), ctypes.POINTER(FgmresOpts), _D, _I, _I,
                                _P, ctypes.POINTER(StepStats)]),
    "dg_device_bytes": (_D, [_P]),
    "dg_footprint_bytes": (_D, [ctypes.POINTER(MeshDesc), _I, ctypes.POINTER(PmgOpts), ctypes.POINTER(FgmresOpts)]),
    "dg_server_create": (_I, [ctypes.POINTER(ServerOpts), ctypes.POINTER(_P)]),
    "dg_server_destroy": (_I, [_P]),
    "dg_server_last_error": (ctypes.c_char_p, [_P]),
    "dg_server_time": (_D, [_P]),
    "dg_server_submit": (_I, [_P, ctypes.POINTER(Request)]),
    "dg_server_poll": (_I, [_P, ctypes.POINTER(Response), _I, _I]),
    "dg_server_drain": (_I, [_P]),
    "dg_server_stats": (_I, [_P, ctypes.POINTER(ServerInfo)]),
}
KIND = {name: i for i, name in enumerate(KERNEL_KINDS)}


def mesh_desc(n, lo, hi):
    md = MeshDesc()
    md.nx, md.ny, md.nz = (int(x) for x in n)
    for d in range(3):
        md.lo[d] = float(lo[d])
        md.hi[d] = float(hi[d])
    return md


def footprint_bytes(n, lo, hi, p, popts, fopts):
    """Device bytes a context of this mesh/degree allocates for one BDF2 step (host arithmetic only)."""
    return float(load().dg_footprint_bytes(ctypes.byref(mesh_desc(n, lo, hi)), int(p), ctypes.byref(popts),
                                           ctypes.byref(fopts)))

_lib = None


def load(path=LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("HIP library %s is not built; run __graft_entry__.build()" % path)
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class DGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


SMOOTH_BJ, SMOOTH_GMRES = 0, 1
CYCLE_V, CYCLE_FMG = 0, 1
COARSEST_BJ, COARSEST_BILU = 0, 1


def pmg_opts(levels, nu_pre=2, nu_post=2, omega=1.0, coarsest_iters=30, prec_fine=DG_FP64,
             prec_coarse=DG_FP64, coarse_matrix_free=1, coarsest_plain=0, smoother=SMOOTH_BJ, cycle=CYCLE_V,
             coarsest_prec=COARSEST_BJ):
    o = PmgOpts()
    o.n_levels = len(levels)
    for i, p in enumerate(levels):
        o.p_level[i] = int(p)
    o.nu_pre, o.nu_post, o.omega, o.coarsest_iters = nu_pre, nu_post, omega, coarsest_iters
    o.prec_fine, o.prec_coarse, o.coarse_matrix_free = prec_fine, prec_coarse, coarse_matrix_free
    o.coarsest_plain, o.smoother, o.cycle, o.coarsest_prec = coarsest_plain, smoother, cycle, coarsest_prec
    return o


def paper_pmg_opts(levels, prec_fine=DG_FP64, prec_coarse=DG_FP64, coarse_matrix_free=2, coarsest_prec=COARSEST_BJ):
    """The paper's preconditioner (Sec. 6, Alg. 1, Table MGSettings): full
    multigrid, GMRES(BJ) smoothers with 10 iterations on the finer levels, a
    30-iteration coarsest GMRES preconditioned by block Jacobi or (as in the
    table) by block ILU(0) in minimum-discarded-fill order."""
    return pmg_opts(levels, nu_pre=10, nu_post=10, coarsest_iters=30, prec_fine=prec_fine, prec_coarse=prec_coarse,
                    coarse_matrix_free=coarse_matrix_free, smoother=SMOOTH_GMRES, cycle=CYCLE_FMG,
                    coarsest_prec=coarsest_prec)


def fgmres_opts(restart=30, rtol=1e-8, max_restarts=20, jvp_exact=1):
    o = FgmresOpts()
    o.restart, o.rtol, o.max_restarts, o.jvp_exact = restart, rtol, max_restarts, jvp_exact
    return o


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One DG discretisation on the current CUDA (HIP) device.

    n: elements per direction; lo, hi: periodic box; p: degree (1..4);
    gamma, mu (0 = Euler), Pr, eta: gas model and BR2 penalty;
    vertices: optional host float64 array (ne, 8, 3) of Q1 vertices."""

    def __init__(self, n, lo, hi, p, gamma=1.4, mu=0.0, Pr=0.72, eta=7.0, vertices=None, stream=None, _borrow=None):
        import numpy as np
        import torch
        self.torch = torch
        self.lib = load()
        self.owned = _borrow is None
        self.sync = not self.owned
        if _borrow is not None:        # a context owned by a Batch (runs on the case's own stream)
            self.h = ctypes.c_void_p(_borrow)
            self.stream = None
            self.n, self.p = tuple(int(x) for x in n), int(p)
            self.ne = self.n[0] * self.n[1] * self.n[2]
            self.nv = (self.p + 1) ** 3
            self.ndof = int(self.lib.dg_ndof(self.h))
            self.device = torch.device("cuda", torch.cuda.current_device())
            return
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        md = MeshDesc()
        md.nx, md.ny, md.nz = (int(x) for x in n)
        for d in range(3):
            md.lo[d] = float(lo[d])
            md.hi[d] = float(hi[d])
        self._vtx = None
        if vertices is not None:
            self._vtx = np.ascontiguousarray(vertices, dtype=np.float64)
            md.vtx = self._vtx.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        ph = Phys(gamma, mu, Pr, eta)
        h = ctypes.c_void_p()
        st = self.lib.dg_create(ctypes.byref(md), ctypes.byref(ph), int(p), ctypes.c_void_p(self.stream.cuda_stream),
                                ctypes.byref(h))
        if st != DG_OK:
            raise DGError(st, "dg_create failed")
        self.h = h
        self.n, self.p = tuple(int(x) for x in n), int(p)
        self.ne = md.nx * md.ny * md.nz
        self.nv = (p + 1) ** 3
        self.ndof = int(self.lib.dg_ndof(h))
        self.device = torch.device("cuda", torch.cuda.current_device())

    # ---- helpers -------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            if self.owned:
                self.lib.dg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != DG_OK:
            raise DGError(st, self.lib.dg_last_error(self.h).decode())
        if self.sync:                  # borrowed context: its stream is not torch's
            self.torch.cuda.synchronize()

    def _vec(self, t, name, n=None):
        torch = self.torch
        if self.sync:                  # borrowed context: inputs written on torch's stream must be ready
            torch.cuda.synchronize()
        n = self.ndof if n is None else n
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
                and t.numel() == n):
            raise ValueError("%s must be a contiguous float64 CUDA tensor with %d entries" % (name, n))
        return _ptr(t)

    def empty(self, n=None):
        return self.torch.empty(self.ndof if n is None else n, dtype=self.torch.float64, device=self.device)

    # ---- entry points ---------------------------------------------------------
    def quad_points(self):
        out = self.empty(self.ne * self.nv * 3)
        self._check(self.lib.dg_quad_points(self.h, _ptr(out)))
        return out.view(self.ne, self.nv, 3)

    def project(self, values, W=None):
        values = values.contiguous()
        self._vec(values, "values", self.ne * self.nv * 5)
        W = self.empty() if W is None else W
        self._check(self.lib.dg_project(self.h, _ptr(values), self._vec(W, "W")))
        return W

    def residual(self, W, R=None):
        R = self.empty() if R is None else R
        self._check(self.lib.dg_residual(self.h, self._vec(W, "W"), self._vec(R, "R")))
        return R

    def jvp(self, W, RW, v, shift, y=None):
        y = self.empty() if y is None else y
        self._check(self.lib.dg_jvp(self.h, self._vec(W, "W"), self._vec(RW, "RW"), self._vec(v, "v"),
                                    float(shift), self._vec(y, "y")))
        return y

    def jvp_exact(self, W, v, shift, y=None):
        y = self.empty() if y is None else y
        self._check(self.lib.dg_jvp_exact(self.h, self._vec(W, "W"), self._vec(v, "v"), float(shift),
                                          self._vec(y, "y")))
        return y

    def mass(self, v, y=None):
        y = self.empty() if y is None else y
        self._check(self.lib.dg_mass(self.h, self._vec(v, "v"), self._vec(y, "y")))
        return y

    def assemble_diag(self, W, shift):
        nb = 5 * self.nv
        out = self.empty(self.ne * nb * nb)
        self._check(self.lib.dg_assemble_diag(self.h, self._vec(W, "W"), float(shift), _ptr(out)))
        return out.view(self.ne, nb, nb)       # [e][col][row]

    def assemble_diag_noalloc(self, W, shift, out):
        """dg_assemble_diag_noalloc into the caller's float64 tensor `out`
        (ne * nb * nb entries): the library allocates nothing."""
        nb = 5 * self.nv
        self._check(self.lib.dg_assemble_diag_noalloc(self.h, self._vec(W, "W"), float(shift),
                                                      self._vec(out, "out", self.ne * nb * nb)))
        return out.view(self.ne, nb, nb)       # [e][col][row]

    def assemble_coarse(self, W, pc):
        nbc = 5 * (pc + 1) ** 3
        out = self.empty(self.ne * 6 * nbc * nbc)
        self._check(self.lib.dg_assemble_coarse(self.h, self._vec(W, "W"), int(pc), _ptr(out)))
        return out.view(self.ne, 6, nbc, nbc)     # [e][f][col][row]

    def assemble_operator(self, W, shift):
        """Store K = shift M + dR/dW at W in the context (7 FP64 blocks per element)."""
        self._check(self.lib.dg_assemble_operator(self.h, self._vec(W, "W"), float(shift)))

    def jvp_assembled(self, v, y=None):
        """y = K v with the operator of the last assemble_operator call."""
        y = self.empty() if y is None else y
        self._check(self.lib.dg_jvp_assembled(self.h, self._vec(v, "v"), self._vec(y, "y")))
        return y

    def pmg_setup(self, W, shift, opts):
        self._check(self.lib.pmg_setup(self.h, self._vec(W, "W"), float(shift), ctypes.byref(opts)))

    def pmg_apply(self, r, z=None):
        z = self.empty() if z is None else z
        self._check(self.lib.pmg_apply(self.h, self._vec(r, "r"), self._vec(z, "z")))
        return z

    def fgmres(self, W, RW, b, opts, x=None, raise_on_noconv=True):
        x = self.empty() if x is None else x
        st = FgmresStats()
        s = self.lib.fgmres_step(self.h, self._vec(W, "W"), self._vec(RW, "RW"), self._vec(b, "b"),
                                 self._vec(x, "x"), ctypes.byref(opts), ctypes.byref(st))
        if s != DG_OK and (raise_on_noconv or s != DG_ENOCONV):
            self._check(s)
        return x, st

    def use_graphs(self, enable):
        self._check(self.lib.dg_use_graphs(self.h, 1 if enable else 0))

    def device_bytes(self):
        return float(self.lib.dg_device_bytes(self.h))

    def timing(self, enable):
        self._check(self.lib.dg_timing(self.h, 1 if enable else 0))

    def timing_read(self):
        """{kernel family: (total device ms, launches, algorithmic bytes, flops)} since the last clear."""
        k = len(KERNEL_KINDS)
        ms = (ctypes.c_double * k)()
        cnt = (ctypes.c_int * k)()
        by = (ctypes.c_double * k)()
        fl = (ctypes.c_double * k)()
        self._check(self.lib.dg_timing_read(self.h, ms, cnt, by, fl))
        return {KERNEL_KINDS[i]: (ms[i], cnt[i], by[i], fl[i]) for i in range(k)}

    def esdirk3_step(self, Wn, dt, popts, fopts, newton_rtol=1e-10, max_newton=5, Wnp1=None):
        Wnp1 = self.empty() if Wnp1 is None else Wnp1
        st = StepStats()
        self._check(self.lib.dg_esdirk3_step(self.h, self._vec(Wn, "Wn"), float(dt), ctypes.byref(popts),
                                             ctypes.byref(fopts), float(newton_rtol), int(max_newton),
                                             self._vec(Wnp1, "Wnp1"), ctypes.byref(st)))
        return Wnp1, st

    def bdf2_step(self, Wn, Wnm1, dt, popts, fopts, newton_rtol=1e-10, max_newton=5, Wnp1=None):
        Wnp1 = self.empty() if Wnp1 is None else Wnp1
        st = StepStats()
        wm = self._vec(Wnm1, "Wnm1") if Wnm1 is not None else None
        self._check(self.lib.dg_bdf2_step(self.h, self._vec(Wn, "Wn"), wm, float(dt), ctypes.byref(popts),
                                          ctypes.byref(fopts), float(newton_rtol), int(max_newton),
                                          self._vec(Wnp1, "Wnp1"), ctypes.byref(st)))
        return Wnp1, st


def batched_lu(A, piv, stream=None):
    """In-place PLU of a (nblk, n, n) float64 CUDA tensor holding column-major blocks."""
    import torch
    lib = load()
    s = stream if stream is not None else torch.cuda.current_stream()
    nblk, n, _ = A.shape
    st = lib.dg_batched_lu(ctypes.c_void_p(s.cuda_stream), _ptr(A), _ptr(piv), nblk, n)
    if st != DG_OK:
        raise DGError(st, "dg_batched_lu")


def batched_lu_solve(LU, piv, b, x, stream=None):
    import torch
    lib = load()
    s = stream if stream is not None else torch.cuda.current_stream()
    nblk, n, _ = LU.shape
    st = lib.dg_batched_lu_solve(ctypes.c_void_p(s.cuda_stream), _ptr(LU), _ptr(piv), _ptr(b), _ptr(x), nblk, n)
    if st != DG_OK:
        raise DGError(st, "dg_batched_lu_solve")


class Batch:
    """Many independent cases on the current device (dg_batch_* entry points).

    cases: list of dicts with keys n, lo, hi, p and optional gamma, mu, Pr,
    eta, vertices.  Batched vectors concatenate the cases' vectors in order;
    `split` returns per-case views."""

    def __init__(self, cases, stream=None):
        import numpy as np
        import torch
        self.torch = torch
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (CaseDesc * len(cases))()
        self._keep = []
        for i, c in enumerate(cases):
            d = arr[i]
            d.mesh.nx, d.mesh.ny, d.mesh.nz = (int(x) for x in c["n"])
            for k in range(3):
                d.mesh.lo[k] = float(c["lo"][k])
                d.mesh.hi[k] = float(c["hi"][k])
            if c.get("vertices") is not None:
                v = np.ascontiguousarray(c["vertices"], dtype=np.float64)
                self._keep.append(v)
                d.mesh.vtx = v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.phys = Phys(c.get("gamma", 1.4), c.get("mu", 0.0), c.get("Pr", 0.72), c.get("eta", 7.0))
            d.p = int(c["p"])
        h = ctypes.c_void_p()
        st = self.lib.dg_batch_create(arr, len(cases), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != DG_OK:
            raise DGError(st, "dg_batch_create failed")
        self.h = h
        self.cases = [dict(c) for c in cases]
        self.nc = len(cases)
        self.ndof = int(self.lib.dg_batch_ndof(h, -1))
        self.sizes = [int(self.lib.dg_batch_ndof(h, i)) for i in range(self.nc)]
        self.offsets = [int(self.lib.dg_batch_offset(h, i)) for i in range(self.nc)]
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "h", None):
            self.lib.dg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, ok=(DG_OK,)):
        if st not in ok:
            raise DGError(st, self.lib.dg_batch_last_error(self.h).decode())
        return st

    def _vec(self, t, name):
        torch = self.torch
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
                and t.numel() == self.ndof):
            raise ValueError("%s must be a contiguous float64 CUDA tensor with %d entries" % (name, self.ndof))
        return _ptr(t)

    def empty(self):
        return self.torch.empty(self.ndof, dtype=self.torch.float64, device=self.device)

    def split(self, t):
        return [t[o:o + n] for o, n in zip(self.offsets, self.sizes)]

    def case(self, c):
        """The case's own context (borrowed: single-context calls on the case's stream)."""
        h = self.lib.dg_batch_case(self.h, int(c))
        cd = self.cases[c]
        return Context(cd["n"], cd["lo"], cd["hi"], cd["p"], _borrow=h)

    def residual(self, W, R=None):
        R = self.empty() if R is None else R
        self._check(self.lib.dg_batch_residual(self.h, self._vec(W, "W"), self._vec(R, "R")))
        return R

    def jvp(self, W, RW, v, shift, y=None):
        y = self.empty() if y is None else y
        self._check(self.lib.dg_batch_jvp(self.h, self._vec(W, "W"), self._vec(RW, "RW"), self._vec(v, "v"),
                                          float(shift), self._vec(y, "y")))
        return y

    def jvp_exact(self, W, v, shift, y=None):
        y = self.empty() if y is None else y
        self._check(self.lib.dg_batch_jvp_exact(self.h, self._vec(W, "W"), self._vec(v, "v"), float(shift),
                                                self._vec(y, "y")))
        return y

    def use_graphs(self, enable):
        self._check(self.lib.dg_batch_use_graphs(self.h, 1 if enable else 0))

    @staticmethod
    def _tile_dict(t):
        return dict(threads=t.threads, epb=list(t.epb)[1:], grid=t.grid, lds_bytes=int(t.lds_bytes), ms=t.ms,
                    candidates=t.candidates, items=t.items)

    def tile(self, kind):
        t = BatchTile()
        self._check(self.lib.dg_batch_get_tile(self.h, KIND[kind], ctypes.byref(t)))
        return self._tile_dict(t)

    def set_tile(self, kind, threads, lds_cap, grid_per_cu):
        self._check(self.lib.dg_batch_set_tile(self.h, KIND[kind], int(threads), int(lds_cap), int(grid_per_cu)))

    def tune(self, kind, W, RW=None, v=None, reps=3):
        t = BatchTile()
        self._check(self.lib.dg_batch_tune(self.h, KIND[kind], self._vec(W, "W"),
                                           self._vec(RW, "RW") if RW is not None else None,
                                           self._vec(v, "v") if v is not None else None, int(reps),
                                           ctypes.byref(t)))
        return self._tile_dict(t)

    def bdf2_step(self, Wn, Wnm1, dt, popts, fopts, newton_rtol=1e-10, max_newton=5, workers=8, Wnp1=None,
                  raise_on_noconv=True):
        """popts: one pmg_opts per case.  Returns (Wnp1, [StepStats], status)."""
        Wnp1 = self.empty() if Wnp1 is None else Wnp1
        po = (PmgOpts * self.nc)(*popts)
        st = (StepStats * self.nc)()
        wm = self._vec(Wnm1, "Wnm1") if Wnm1 is not None else None
        s = self.lib.dg_batch_bdf2_step(self.h, self._vec(Wn, "Wn"), wm, float(dt), po, ctypes.byref(fopts),
                                        float(newton_rtol), int(max_newton), int(workers), self._vec(Wnp1, "Wnp1"),
                                        st)
        self._check(s, (DG_OK,) if raise_on_noconv else (DG_OK, DG_ENOCONV))
        return Wnp1, list(st), s


class Server:
    """Serving loop (dg_server_*): submit BDF2 step requests, poll responses.

    Inputs must be complete on the device before submit (the step runs on a
    stream of its own); keep the tensors alive until the response is polled."""

    def __init__(self, slots=4, hbm_budget=0.0, cache=True):
        import torch
        self.torch = torch
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible")
        o = ServerOpts(int(slots), float(hbm_budget), 1 if cache else 0)
        h = ctypes.c_void_p()
        st = self.lib.dg_server_create(ctypes.byref(o), ctypes.byref(h))
        if st != DG_OK:
            raise DGError(st, "dg_server_create failed")
        self.h = h
        self._keep = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.dg_server_destroy(self.h)
            self.h = None
            self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def time(self):
        return float(self.lib.dg_server_time(self.h))

    def submit(self, tag, n, lo, hi, p, Wn, Wnp1, dt, popts, fopts, gamma=1.4, mu=0.0, Pr=0.72, eta=7.0,
               Wnm1=None, newton_rtol=1e-10, max_newton=5):
        rq = Request()
        rq.mesh = mesh_desc(n, lo, hi)
        rq.phys = Phys(gamma, mu, Pr, eta)
        rq.p, rq.dt, rq.popts, rq.fopts = int(p), float(dt), popts, fopts
        rq.newton_rtol, rq.max_newton = float(newton_rtol), int(max_newton)
        rq.Wn, rq.Wnp1 = Wn.data_ptr(), Wnp1.data_ptr()
        rq.Wnm1 = Wnm1.data_ptr() if Wnm1 is not None else None
        rq.tag = int(tag)
        st = self.lib.dg_server_submit(self.h, ctypes.byref(rq))
        if st != DG_OK:
            raise DGError(st, "dg_server_submit failed")
        self._keep[int(tag)] = (Wn, Wnp1, Wnm1)

    def poll(self, max_n=256, wait_ms=0):
        buf = (Response * max_n)()
        k = self.lib.dg_server_poll(self.h, buf, int(max_n), int(wait_ms))
        if k < 0:
            raise DGError(DG_EINVAL, "dg_server_poll failed")
        out = [buf[i] for i in range(k)]
        for r in out:
            self._keep.pop(int(r.tag), None)
        return out

    def drain(self):
        st = self.lib.dg_server_drain(self.h)
        if st != DG_OK:
            raise DGError(st, "dg_server_drain failed")

    def info(self):
        i = ServerInfo()
        self.lib.dg_server_stats(self.h, ctypes.byref(i))
        return dict(submitted=i.submitted, completed=i.completed, pending=i.pending, running=i.running,
                    contexts=i.contexts, held_bytes=i.held_bytes, peak_held_bytes=i.peak_held_bytes,
                    budget_bytes=i.budget_bytes)

    def last_error(self):
        return self.lib.dg_server_last_error(self.h).decode()
