"""Python binding of the C ABI in include/seedcg.h (ctypes; argument marshalling only).

Every array is a torch tensor on the GPU in the canonical layouts of the C ABI:
  links (4, V, 3, 3) complex128, vectors (n, Vh, 4, 3) complex128, contiguous.
All arithmetic runs in the HIP library; if libseedcg.so is missing this module raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libseedcg.so")

FP64, MIXED_FP32, MIXED_FP32_BF16LINKS, MIXED_FP32_CG = 0, 1, 2, 3
_PREC = {"fp64": FP64, "mixed": MIXED_FP32, "mixed_fp32": MIXED_FP32, "mixed_bf16": MIXED_FP32_BF16LINKS,
         "mixed_cg": MIXED_FP32_CG}
STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_OOM", -3: "ERR_HIP", -4: "ERR_BREAKDOWN", -5: "ERR_NOCONV",
          -6: "ERR_STATE"}
SEED_STATUS = {0: "ok", 1: "breakdown", 2: "indefinite", 3: "capped"}


class Params(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("kappa", ctypes.c_double), ("t_bc", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("m_max", ctypes.c_int32), ("reorth_k", ctypes.c_int32),
                ("past_factor", ctypes.c_double), ("tol", ctypes.c_double), ("reliable_every", ctypes.c_int32),
                ("seed_block", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("deflate", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("basis_fp32", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("iters", ctypes.POINTER(ctypes.c_int32)), ("matvecs", ctypes.POINTER(ctypes.c_int32)),
                ("true_relres", ctypes.POINTER(ctypes.c_double)), ("m_used", ctypes.c_int32),
                ("i_conv", ctypes.c_int32), ("seed_status", ctypes.c_int32), ("reorth_passes", ctypes.c_int32),
                ("t_seed_s", ctypes.c_double), ("t_rest_s", ctypes.c_double),
                ("est_relres", ctypes.POINTER(ctypes.c_double)), ("orth_loss_max", ctypes.c_double),
                ("t_train_s", ctypes.c_double)]


class SeedCGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Load libseedcg.so (built by paper_0901_3512_amd.build); raises if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_0901_3512_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    H = ctypes.c_void_p
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "seedcg_default_params": (None, [ctypes.POINTER(Params)]),
        "seedcg_create": (i32, [ctypes.POINTER(Params), P, ctypes.POINTER(H)]),
        "seedcg_apply_M": (i32, [H, P, P, i32]),
        "seedcg_apply_M_inner": (i32, [H, P, P, i32]),
        "seedcg_apply_A": (i32, [H, P, P, i32, i32]),
        "seedcg_solve_seed": (i32, [H, P, P, i32, ctypes.POINTER(Report)]),
        "seedcg_solve_rest": (i32, [H, P, P, i32, ctypes.POINTER(Report)]),
        "seedcg_solve_repeated": (i32, [H, P, P, i32, ctypes.POINTER(Report)]),
        "seedcg_solve_indefinite": (i32, [H, P, P, i32, ctypes.POINTER(Report)]),
        "seedcg_get_tridiag": (i32, [H, ctypes.POINTER(dbl), ctypes.POINTER(dbl), i32, ctypes.POINTER(i32)]),
        "seedcg_get_basis_vector": (i32, [H, i32, P]),
        "seedcg_get_ritz": (i32, [H, ctypes.POINTER(dbl), i32, ctypes.POINTER(i32)]),
        "seedcg_project": (i32, [H, P, i32, P, i32, i64, P]),
        "seedcg_project_noalloc": (i32, [H, P, i32, P, i32, i64, P]),
        "seedcg_update": (i32, [H, P, i32, P, P, i32, i64]),
        "seedcg_train_precond": (i32, [H, i32, i32, i32, dbl, ctypes.POINTER(dbl)]),
        "seedcg_use_precond": (i32, [H, i32]),
        "seedcg_set_precond_weights": (i32, [H, ctypes.POINTER(dbl)]),
        "seedcg_get_precond_weights": (i32, [H, ctypes.POINTER(dbl)]),
        "seedcg_apply_P": (i32, [H, P, P, i32]),
        "seedcg_precond_loss_grad": (i32, [H, P, P, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]),
        "seedcg_precond_loss_grad_band": (i32, [H, P, P, i32, i32, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]),
        "seedcg_set_timing": (i32, [H, i32, i32]),
        "seedcg_get_timing": (i32, [H, ctypes.POINTER(dbl)]),
        "seedcg_get_timing_kinds": (i32, [H, ctypes.POINTER(dbl), i32, ctypes.POINTER(i32)]),
        "seedcg_time_M": (i32, [H, i32, i32, i32, ctypes.POINTER(dbl)]),
        "seedcg_probe_bandwidth": (i32, [i32, i64, i32, P, ctypes.POINTER(dbl)]),
        "seedcg_probe_mfma": (i32, [i32, i32, P, ctypes.POINTER(dbl)]),
        "seedcg_release_basis": (i32, [H]),
        "seedcg_destroy": (None, [H]),
        "seedcg_last_error": (ctypes.c_char_p, [H]),
        "seedcg_create_batch": (i32, [i32, ctypes.POINTER(i32), ctypes.POINTER(dbl), ctypes.POINTER(P), i32,
                                      ctypes.POINTER(Params), ctypes.POINTER(H)]),
        "seedcg_solve_batch": (i32, [H, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(Report)]),
        "seedcg_batch_info": (i32, [H, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(dbl)]),
        "seedcg_batch_set_timing": (i32, [H, i32, i32]),
        "seedcg_batch_get_timing": (i32, [H, ctypes.POINTER(dbl)]),
        "seedcg_destroy_batch": (None, [H]),
        "seedcg_batch_last_error": (ctypes.c_char_p, [H]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names of the C ABI entry points this binding expects."""
    return ["seedcg_default_params", "seedcg_create", "seedcg_apply_M", "seedcg_apply_M_inner", "seedcg_apply_A", "seedcg_solve_seed",
            "seedcg_solve_rest", "seedcg_solve_repeated", "seedcg_solve_indefinite", "seedcg_get_tridiag", "seedcg_get_basis_vector", "seedcg_get_ritz", "seedcg_project",
            "seedcg_project_noalloc", "seedcg_update", "seedcg_train_precond", "seedcg_use_precond", "seedcg_set_precond_weights",
            "seedcg_get_precond_weights", "seedcg_apply_P", "seedcg_precond_loss_grad", "seedcg_precond_loss_grad_band", "seedcg_set_timing",
            "seedcg_get_timing", "seedcg_get_timing_kinds", "seedcg_time_M", "seedcg_probe_bandwidth", "seedcg_probe_mfma", "seedcg_release_basis", "seedcg_destroy", "seedcg_last_error", "seedcg_create_batch",
            "seedcg_solve_batch", "seedcg_batch_info", "seedcg_batch_set_timing", "seedcg_batch_get_timing",
            "seedcg_destroy_batch", "seedcg_batch_last_error"]


_PROBE_KINDS = {"copy": 0, "triad": 1, "read": 2}


def probe_bandwidth(kind, nbytes=1 << 31, reps=10, stream=None):
    """GB/s this GPU reaches with the library's copy, FP64 triad or read kernel over buffers of nbytes
    each (every byte read or written counted once); a roofline probe, not part of the method."""
    lib = load_library()
    if stream is None:
        stream = torch.cuda.current_stream()
    out = ctypes.c_double()
    rc = lib.seedcg_probe_bandwidth(_PROBE_KINDS[kind], int(nbytes), int(reps), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(out))
    if rc != 0:
        raise SeedCGError(rc, lib.seedcg_last_error(None).decode())
    return out.value


def probe_mfma(dtype="fp64", iters=20000, stream=None):
    """TFLOP/s of register-resident v_mfma_f64_16x16x4 (dtype "fp64") or v_mfma_f32_16x16x4 ("fp32")
    chains on every SIMD; a roofline probe, not part of the method."""
    lib = load_library()
    if stream is None:
        stream = torch.cuda.current_stream()
    out = ctypes.c_double()
    rc = lib.seedcg_probe_mfma({"fp64": 0, "fp32": 1}[dtype], int(iters), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(out))
    if rc != 0:
        raise SeedCGError(rc, lib.seedcg_last_error(None).decode())
    return out.value


def _check_vec(t, Vh, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name}: expected a complex128 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.dim() == 3:
        t = t.unsqueeze(0)
    if tuple(t.shape[1:]) != (Vh, 4, 3):
        raise ValueError(f"{name}: expected shape (n, {Vh}, 4, 3), got {tuple(t.shape)}")
    return t


class SeedCG:
    """One gauge configuration: M = A^dag A with A = 1 - kappa^2 H_eo H_oe (see include/seedcg.h)."""

    def __init__(self, links, dims, kappa, *, t_bc=-1, prec="fp64", m_max=0, reorth_k=10, past=1.5,
                 tol=1e-10, reliable_every=50, seed_block=32, max_iter=100000, autotune=True, deflate=0, basis_fp32=False,
                 stream=None):
        lib = load_library()
        self.dims = tuple(int(d) for d in dims)
        self.V = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        self.Vh = self.V // 2
        if not (isinstance(links, torch.Tensor) and links.is_cuda and links.dtype == torch.complex128):
            raise TypeError("links: expected a complex128 CUDA tensor")
        if tuple(links.shape) != (4, self.V, 3, 3) or not links.is_contiguous():
            raise ValueError(f"links: expected a contiguous (4, {self.V}, 3, 3) tensor")
        self.device = links.device
        p = Params()
        lib.seedcg_default_params(ctypes.byref(p))
        for d in range(4):
            p.dims[d] = self.dims[d]
        p.kappa = float(kappa)
        p.t_bc = int(t_bc)
        p.prec = _PREC[prec] if isinstance(prec, str) else int(prec)
        p.m_max = int(m_max)
        p.reorth_k = int(reorth_k)
        p.past_factor = float(past)
        p.tol = float(tol)
        p.reliable_every = int(reliable_every)
        p.seed_block = int(seed_block)
        p.max_iter = int(max_iter)
        p.autotune = int(bool(autotune))
        p.deflate = int(deflate)
        # False / True / "reorth": FP64 basis; FP32 basis; FP64 basis plus an FP32 copy read only by
        # the reorthogonalisation
        p.basis_fp32 = 2 if basis_fp32 == "reorth" else int(bool(basis_fp32))
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        p.stream = ctypes.c_void_p(stream.cuda_stream)
        self.params = p
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib.seedcg_create(ctypes.byref(p), ctypes.c_void_p(links.data_ptr()), ctypes.byref(h))
        if rc != 0:
            raise SeedCGError(rc, lib.seedcg_last_error(None).decode())
        self._h = h
        self._lib = lib

    # -- helpers -----------------------------------------------------------------------------
    def _rc(self, rc):
        if rc != 0:
            raise SeedCGError(rc, self._lib.seedcg_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            self._lib.seedcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C ABI calls ---------------------------------------------------------------------------
    def apply_M(self, x):
        x = _check_vec(x, self.Vh, "x")
        y = torch.empty_like(x)
        self._rc(self._lib.seedcg_apply_M(self._h, x.data_ptr(), y.data_ptr(), x.shape[0]))
        return y

    def apply_M_inner(self, x):
        """M x with the solver's inner precision (FP32/BF16 links for the mixed modes)."""
        x = _check_vec(x, self.Vh, "x")
        y = torch.empty_like(x)
        self._rc(self._lib.seedcg_apply_M_inner(self._h, x.data_ptr(), y.data_ptr(), x.shape[0]))
        return y

    def apply_A(self, x, dagger=False):
        x = _check_vec(x, self.Vh, "x")
        y = torch.empty_like(x)
        self._rc(self._lib.seedcg_apply_A(self._h, x.data_ptr(), y.data_ptr(), x.shape[0], int(bool(dagger))))
        return y

    def _report(self, n):
        it = (ctypes.c_int32 * n)()
        mv = (ctypes.c_int32 * n)()
        rr = (ctypes.c_double * n)()
        r = Report()
        r.iters = ctypes.cast(it, ctypes.POINTER(ctypes.c_int32))
        r.matvecs = ctypes.cast(mv, ctypes.POINTER(ctypes.c_int32))
        r.true_relres = ctypes.cast(rr, ctypes.POINTER(ctypes.c_double))
        r._est = (ctypes.c_double * n)()   # kept alive with the report
        r.est_relres = ctypes.cast(r._est, ctypes.POINTER(ctypes.c_double))
        return r, it, mv, rr

    def solve_seed(self, B, X=None):
        """Algorithm 1; returns (X, report).  X[0]: RHS-1 iterate, X[1:]: seeded guesses."""
        B = _check_vec(B, self.Vh, "B")
        X = torch.zeros_like(B) if X is None else _check_vec(X, self.Vh, "X")
        n = B.shape[0]
        r, it, mv, rr = self._report(n)
        self._rc(self._lib.seedcg_solve_seed(self._h, B.data_ptr(), X.data_ptr(), n, ctypes.byref(r)))
        rep = dict(m=r.m_used, i_conv=r.i_conv, seed_status=SEED_STATUS.get(r.seed_status, r.seed_status),
                   reorth_passes=r.reorth_passes, t_seed_s=r.t_seed_s, matvecs=list(mv), est_relres=list(r._est),
                   orth_loss_max=r.orth_loss_max)
        return X, rep

    def solve_rest(self, B, X, raise_on_noconv=True):
        """Plain CG from X on every right-hand side above tol; returns (X, report)."""
        B = _check_vec(B, self.Vh, "B")
        X = _check_vec(X, self.Vh, "X")
        n = B.shape[0]
        r, it, mv, rr = self._report(n)
        rc = self._lib.seedcg_solve_rest(self._h, B.data_ptr(), X.data_ptr(), n, ctypes.byref(r))
        rep = dict(iters=list(it), matvecs=list(mv), true_relres=list(rr), t_rest_s=r.t_rest_s,
                   est_relres=list(r._est), t_train_s=r.t_train_s, status=STATUS.get(rc, rc))
        if rc != 0 and (rc != -5 or raise_on_noconv):
            self._rc(rc)
        return X, rep

    def solve_repeated(self, B, X=None, raise_on_noconv=True):
        """Traditional repeated seeding, then CG where needed; returns (X, report)."""
        B = _check_vec(B, self.Vh, "B")
        X = torch.zeros_like(B) if X is None else _check_vec(X, self.Vh, "X")
        n = B.shape[0]
        r, it, mv, rr = self._report(n)
        rc = self._lib.seedcg_solve_repeated(self._h, B.data_ptr(), X.data_ptr(), n, ctypes.byref(r))
        rep = dict(iters=list(it), matvecs=list(mv), true_relres=list(rr), m=r.m_used, i_conv=r.i_conv,
                   status=STATUS.get(rc, rc))
        if rc != 0 and (rc != -5 or raise_on_noconv):
            self._rc(rc)
        return X, rep

    def solve_indefinite(self, Phi, X=None, raise_on_noconv=True):
        """A x = phi through H = gamma5 A: seeded Lanczos with the QR (MINRES) factorisation, then
        MINRES; Phi holds the right-hand sides phi (not A^dag phi).  Returns (X, report)."""
        Phi = _check_vec(Phi, self.Vh, "Phi")
        X = torch.zeros_like(Phi) if X is None else _check_vec(X, self.Vh, "X")
        n = Phi.shape[0]
        r, it, mv, rr = self._report(n)
        rc = self._lib.seedcg_solve_indefinite(self._h, Phi.data_ptr(), X.data_ptr(), n, ctypes.byref(r))
        rep = dict(iters=list(it), matvecs=list(mv), true_relres=list(rr), m=r.m_used, i_conv=r.i_conv,
                   seed_status=r.seed_status, reorth_passes=r.reorth_passes, t_seed_s=r.t_seed_s, t_rest_s=r.t_rest_s,
                   status=STATUS.get(rc, rc))
        if rc != 0 and (rc != -5 or raise_on_noconv):
            self._rc(rc)
        return X, rep

    def get_tridiag(self):
        m = ctypes.c_int32()
        self._rc(self._lib.seedcg_get_tridiag(self._h, None, None, 0, ctypes.byref(m)))
        n = m.value
        a = (ctypes.c_double * max(n, 1))()
        b = (ctypes.c_double * (n + 1))()
        self._rc(self._lib.seedcg_get_tridiag(self._h, a, b, n, ctypes.byref(m)))
        return list(a)[:n], list(b)[:n + 1]

    def get_ritz(self):
        """Ritz values of the deflation space used by the last deflated solve_rest (ascending)."""
        n = ctypes.c_int32()
        self._rc(self._lib.seedcg_get_ritz(self._h, None, 0, ctypes.byref(n)))
        th = (ctypes.c_double * max(n.value, 1))()
        self._rc(self._lib.seedcg_get_ritz(self._h, th, n.value, ctypes.byref(n)))
        return list(th)[:n.value]

    def get_basis_vector(self, i):
        v = torch.empty((1, self.Vh, 4, 3), dtype=torch.complex128, device=self.device)
        self._rc(self._lib.seedcg_get_basis_vector(self._h, int(i), v.data_ptr()))
        return v[0]

    def project(self, Vv, R):
        """P = V^dag R for flat complex128 (nv, n) and (nr, n) CUDA tensors."""
        Vv = Vv.reshape(Vv.shape[0], -1)
        R = R.reshape(R.shape[0], -1)
        assert Vv.is_contiguous() and R.is_contiguous() and Vv.shape[1] == R.shape[1]
        P = torch.empty((Vv.shape[0], R.shape[0]), dtype=torch.complex128, device=self.device)
        self._rc(self._lib.seedcg_project(self._h, Vv.data_ptr(), Vv.shape[0], R.data_ptr(), R.shape[0],
                                          Vv.shape[1], P.data_ptr()))
        return P

    def project_noalloc(self, Vv, R, P=None):
        """seedcg_project_noalloc: P = V^dag R with the partials in the library's static device array
        (no allocation inside the library; P may be passed in to avoid torch's too)."""
        Vv = Vv.reshape(Vv.shape[0], -1)
        R = R.reshape(R.shape[0], -1)
        assert Vv.is_contiguous() and R.is_contiguous() and Vv.shape[1] == R.shape[1]
        if P is None:
            P = torch.empty((Vv.shape[0], R.shape[0]), dtype=torch.complex128, device=self.device)
        assert P.is_contiguous() and tuple(P.shape) == (Vv.shape[0], R.shape[0]) and P.dtype == torch.complex128
        self._rc(self._lib.seedcg_project_noalloc(self._h, Vv.data_ptr(), Vv.shape[0], R.data_ptr(), R.shape[0],
                                                  Vv.shape[1], P.data_ptr()))
        return P

    def update(self, W, E, X):
        """X += W E for flat complex128 W (nw, n), E (nw, nx), X (nx, n) CUDA tensors (in place)."""
        assert W.is_contiguous() and E.is_contiguous() and X.is_contiguous()
        self._rc(self._lib.seedcg_update(self._h, W.data_ptr(), W.shape[0], E.data_ptr(), X.data_ptr(),
                                         X.shape[0], W.shape[1]))
        return X

    # -- learned preconditioner P = K K^dag -------------------------------------------------------
    def train_precond(self, steps=2000, n_ritz=4, n_lanczos=12, lr=2e-4):
        out = (ctypes.c_double * 22)()
        self._rc(self._lib.seedcg_train_precond(self._h, int(steps), int(n_ritz), int(n_lanczos), float(lr), out))
        return dict(loss0=out[0], loss1=out[1], t_train_s=out[2], n_ritz=int(out[3]), n_train=int(out[4]),
                    accepted=bool(out[5]), judge_s=dict(cg=out[6], start=out[7], trained=out[8]),
                    judge_iters=dict(cg=int(out[9]), start=int(out[10]), trained=int(out[11]), cg_no_deflation=int(out[18])),
                    choice=["plain_cg", "start_K", "trained_K"][int(out[12])],
                    batch_s=dict(M=out[13], P=out[14], deflation=out[20]),
                    predicted_s=dict(cg=out[15], start=out[16], trained=out[17], cg_no_deflation=out[19]),
                    plain_cg_deflates=bool(out[21]))

    def use_precond(self, on=True):
        self._rc(self._lib.seedcg_use_precond(self._h, int(bool(on))))

    def set_precond_weights(self, W):
        import numpy as np
        w = np.ascontiguousarray(np.asarray(W, dtype=np.complex128).reshape(3, 9, 4, 4))
        self._rc(self._lib.seedcg_set_precond_weights(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def get_precond_weights(self):
        import numpy as np
        w = np.empty((3, 9, 4, 4), dtype=np.complex128)
        self._rc(self._lib.seedcg_get_precond_weights(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return w

    def apply_P(self, x):
        x = _check_vec(x, self.Vh, "x")
        y = torch.empty_like(x)
        self._rc(self._lib.seedcg_apply_P(self._h, x.data_ptr(), y.data_ptr(), x.shape[0]))
        return y

    def precond_loss_grad(self, U, Y, band=None):
        """The training loss and its Wirtinger gradient; band = (t0, nt) takes the loss on those t-slices."""
        import numpy as np
        U = _check_vec(U, self.Vh, "U")
        Y = _check_vec(Y, self.Vh, "Y")
        loss = ctypes.c_double()
        g = np.empty((3, 9, 4, 4), dtype=np.complex128)
        t0, nt = band if band else (0, 0)
        self._rc(self._lib.seedcg_precond_loss_grad_band(self._h, U.data_ptr(), Y.data_ptr(), U.shape[0], int(t0), int(nt),
                                                         ctypes.byref(loss), g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return loss.value, g

    def set_timing(self, sample_every, max_samples=4096):
        self._rc(self._lib.seedcg_set_timing(self._h, int(sample_every), int(max_samples)))

    def get_timing(self):
        """Sampled stencil launches: dict(launches, ms, bytes, flops, seen, seen_bytes); seen and
        seen_bytes count every stencil launch issued since set_timing."""
        out = (ctypes.c_double * 6)()
        self._rc(self._lib.seedcg_get_timing(self._h, out))
        return dict(launches=int(out[0]), ms=out[1], bytes=out[2], flops=out[3], seen=int(out[4]), seen_bytes=out[5])

    def get_timing_kinds(self):
        """Sampled stencil launches by kind: list of dict(fmt, nvec, fused, tps, vb, launches, ms, bytes)."""
        cap = 64
        out = (ctypes.c_double * (8 * cap))()
        n = ctypes.c_int32()
        self._rc(self._lib.seedcg_get_timing_kinds(self._h, out, cap, ctypes.byref(n)))
        keys = ("fmt", "nvec", "fused", "tps", "vb", "launches", "ms", "bytes")
        return [dict(zip(keys, [out[8 * k + q] for q in range(8)])) for k in range(min(n.value, cap))]

    def time_M(self, inner=False, nvec=1, reps=200):
        """Back-to-back applications of M timed with events: dict(ms, bytes, bytes_18real, fmt)."""
        out = (ctypes.c_double * 4)()
        self._rc(self._lib.seedcg_time_M(self._h, int(bool(inner)), int(nvec), int(reps), out))
        return dict(ms=out[0], bytes=out[1], bytes_18real=out[2], fmt=int(out[3]))

    def release_basis(self):
        self._rc(self._lib.seedcg_release_basis(self._h))


class SeedCGBatch:
    """Many configurations (any mix of lattice shapes), nrhs right-hand sides each, solved together:
    per configuration Algorithm 1 on its first right-hand side and plain CG on all of them."""

    def __init__(self, links, dims, kappas, nrhs, *, t_bc=-1, prec="mixed", m_max=0, reorth_k=10, past=1.5,
                 tol=1e-10, reliable_every=50, seed_block=32, max_iter=100000, autotune=True, stream=None):
        lib = load_library()
        n = len(links)
        if not (len(dims) == n and len(kappas) == n) or n < 1:
            raise ValueError("links, dims and kappas must have one entry per configuration")
        self.dims = [tuple(int(d) for d in dd) for dd in dims]
        self.Vh = [dd[0] * dd[1] * dd[2] * dd[3] // 2 for dd in self.dims]
        for c, (U, dd) in enumerate(zip(links, self.dims)):
            V = 2 * self.Vh[c]
            if not (isinstance(U, torch.Tensor) and U.is_cuda and U.dtype == torch.complex128):
                raise TypeError(f"links[{c}]: expected a complex128 CUDA tensor")
            if tuple(U.shape) != (4, V, 3, 3) or not U.is_contiguous():
                raise ValueError(f"links[{c}]: expected a contiguous (4, {V}, 3, 3) tensor")
        self.n, self.nrhs = n, int(nrhs)
        self.device = links[0].device
        p = Params()
        lib.seedcg_default_params(ctypes.byref(p))
        p.t_bc = int(t_bc)
        p.prec = _PREC[prec] if isinstance(prec, str) else int(prec)
        p.m_max = int(m_max)
        p.reorth_k = int(reorth_k)
        p.past_factor = float(past)
        p.tol = float(tol)
        p.reliable_every = int(reliable_every)
        p.seed_block = int(seed_block)
        p.max_iter = int(max_iter)
        p.autotune = int(bool(autotune))
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        p.stream = ctypes.c_void_p(stream.cuda_stream)
        dims_a = (ctypes.c_int32 * (4 * n))(*[d for dd in self.dims for d in dd])
        kap_a = (ctypes.c_double * n)(*[float(k) for k in kappas])
        lk_a = (ctypes.c_void_p * n)(*[U.data_ptr() for U in links])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib.seedcg_create_batch(n, dims_a, kap_a, lk_a, self.nrhs, ctypes.byref(p), ctypes.byref(h))
        if rc != 0:
            raise SeedCGError(rc, lib.seedcg_batch_last_error(None).decode())
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.seedcg_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        ncls = ctypes.c_int32()
        self._lib.seedcg_batch_info(self._h, ctypes.byref(ncls), None, None, None)
        k = ncls.value
        cls = (ctypes.c_int32 * self.n)()
        mc = (ctypes.c_int32 * k)()
        tune = (ctypes.c_double * (4 * k))()
        self._lib.seedcg_batch_info(self._h, None, cls, mc, tune)
        return dict(nclass=k, class_of=list(cls), m_cap=list(mc),
                    tune=[tuple(int(x) for x in tune[4 * i:4 * i + 4]) for i in range(k)])

    def set_timing(self, sample_every, max_samples=4096):
        rc = self._lib.seedcg_batch_set_timing(self._h, int(sample_every), int(max_samples))
        if rc != 0:
            raise SeedCGError(rc, self._lib.seedcg_batch_last_error(self._h).decode())

    def get_timing(self):
        """Sampled stencil launches over every shape class: dict(launches, ms, bytes, flops, seen,
        seen_bytes), totals over the classes."""
        out = (ctypes.c_double * 6)()
        rc = self._lib.seedcg_batch_get_timing(self._h, out)
        if rc != 0:
            raise SeedCGError(rc, self._lib.seedcg_batch_last_error(self._h).decode())
        return dict(launches=int(out[0]), ms=out[1], bytes=out[2], flops=out[3], seen=int(out[4]), seen_bytes=out[5])

    def solve(self, B, X=None, raise_on_noconv=True):
        """B: list of (nrhs, Vh_c, 4, 3) complex128 CUDA tensors; returns (X list, per-config reports)."""
        if len(B) != self.n:
            raise ValueError("B: one tensor per configuration")
        B = [_check_vec(b, self.Vh[c], f"B[{c}]") for c, b in enumerate(B)]
        for c, b in enumerate(B):
            if b.shape[0] != self.nrhs:
                raise ValueError(f"B[{c}]: expected {self.nrhs} vectors")
        X = [torch.zeros_like(b) for b in B] if X is None else [_check_vec(x, self.Vh[c], f"X[{c}]") for c, x in enumerate(X)]
        bp = (ctypes.c_void_p * self.n)(*[b.data_ptr() for b in B])
        xp = (ctypes.c_void_p * self.n)(*[x.data_ptr() for x in X])
        reps = (Report * self.n)()
        keep = []
        for c in range(self.n):
            it = (ctypes.c_int32 * self.nrhs)()
            mv = (ctypes.c_int32 * self.nrhs)()
            rr = (ctypes.c_double * self.nrhs)()
            reps[c].iters = ctypes.cast(it, ctypes.POINTER(ctypes.c_int32))
            reps[c].matvecs = ctypes.cast(mv, ctypes.POINTER(ctypes.c_int32))
            reps[c].true_relres = ctypes.cast(rr, ctypes.POINTER(ctypes.c_double))
            keep.append((it, mv, rr))
        rc = self._lib.seedcg_solve_batch(self._h, bp, xp, reps)
        out = []
        for c in range(self.n):
            it, mv, rr = keep[c]
            r = reps[c]
            out.append(dict(iters=list(it), matvecs=list(mv), true_relres=list(rr), m=r.m_used, i_conv=r.i_conv,
                            seed_status=SEED_STATUS.get(r.seed_status, r.seed_status), reorth_passes=r.reorth_passes,
                            t_seed_s=r.t_seed_s, t_rest_s=r.t_rest_s))
        if rc != 0 and (rc != -5 or raise_on_noconv):
            raise SeedCGError(rc, self._lib.seedcg_batch_last_error(self._h).decode())
        return X, out
