"""MI355X-native multi-sphere T-matrix solver (CELES method, arXiv:1706.02145).

Thin Python binding over the C ABI of libceles_amd.so (include/celes.h):
every computation runs in the library's HIP kernels and host C++ code; this
module only converts arguments.  PyTorch is used only to hand device buffers
and streams to the device-pointer entry points.
"""
import ctypes as C

import numpy as np

from ._capi import (CELES_CUBOID_AUTO, CELES_TRANSLATION_DIRECT, CELES_TRANSLATION_ROTATE, CELES_FP64, CELES_HANKEL_DIRECT, CELES_HANKEL_LUT, CELES_MIXED, CELES_SOLVER_BICGSTAB,
                    CELES_SOLVER_GMRES, ERRORS, Options, SolveInfo, lib, LIB_PATH)

__all__ = ["Problem", "Batch", "Network", "CelesError", "default_options", "plan_preconditioner", "mie_coefficients", "translation_tables", "version",
           "s11",
           "CELES_FP64", "CELES_MIXED", "CELES_HANKEL_LUT", "CELES_HANKEL_DIRECT", "CELES_SOLVER_GMRES",
           "CELES_SOLVER_BICGSTAB", "LIB_PATH"]


class CelesError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc, h=None):
    if rc != 0:
        msg = lib().celes_last_error(h)
        raise CelesError(rc, msg.decode() if msg else "")


def version():
    return lib().celes_version()


def default_options(**kw):
    o = Options()
    lib().celes_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def plan_preconditioner(positions, lmax, target_Nj=100.0, mem_cap_bytes=0.0):
    """Budgeted cuboid edge on the host (celes_plan_preconditioner): returns
    (edge, cuboids, bytes, largest cuboid's sphere count)."""
    pos = np.ascontiguousarray(positions, dtype=np.float64)
    e, nb, by, mx = C.c_double(), C.c_int64(), C.c_double(), C.c_int64()
    _check(lib().celes_plan_preconditioner(pos.shape[0], _dptr(pos), int(lmax), float(target_Nj),
                                           float(mem_cap_bytes), C.byref(e), C.byref(nb), C.byref(by),
                                           C.byref(mx)))
    return e.value, nb.value, by.value, mx.value


def mie_coefficients(lmax, kR, m):
    """Q[tau-1, l-1] of one sphere (celes_mie_coefficients)."""
    out = np.zeros(4 * lmax)
    _check(lib().celes_mie_coefficients(lmax, float(kR), float(np.real(m)), float(np.imag(m)), _dptr(out)))
    z = out[0::2] + 1j * out[1::2]
    return z.reshape(2, lmax)


def translation_tables(lmax):
    """(a5, Im b5) arrays indexed [l-1, m+L, l'-1, m'+L, p] (celes_translation_tables)."""
    W = 2 * lmax + 1
    a = np.zeros((lmax, W, lmax, W, W))
    b = np.zeros_like(a)
    _check(lib().celes_translation_tables(lmax, _dptr(a), _dptr(b)))
    return a, b


def _stream_ptr(stream):
    if stream is None:
        return None
    return C.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def s11(problems, theta, n_phi=64):
    """Phase-function element S11(theta): |F|^2 averaged over the solved
    right-hand sides of `problems` and over n_phi azimuths (celes_s11),
    unnormalised."""
    probs = list(problems)
    th = np.ascontiguousarray(np.atleast_1d(theta), dtype=np.float64)
    out = np.zeros(th.size)
    arr = (C.c_void_p * len(probs))(*[p._h.value for p in probs])
    rc = lib().celes_s11(arr, len(probs), th.size, _dptr(th), int(n_phi), _dptr(out))
    if rc != 0:
        raise CelesError(rc, "a problem has no solution" if rc == -10 else "invalid arguments to celes_s11")
    return out


class Problem:
    """One sphere ensemble on one device (celes_create ... celes_destroy)."""

    def __init__(self, positions, radii, n_sphere, n0, wavelength, lmax, options=None, **kw):
        pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
        rad = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
        ns = np.ascontiguousarray(np.broadcast_to(np.asarray(n_sphere, dtype=np.complex128), rad.shape))
        nsv = np.ascontiguousarray(np.stack([ns.real, ns.imag], -1))
        opt = options if options is not None else default_options(**kw)
        self._h = C.c_void_p()
        rc = lib().celes_create(C.byref(self._h), pos.shape[0], _dptr(pos), _dptr(rad), _dptr(nsv), float(n0),
                                float(wavelength), int(lmax), C.byref(opt))
        if rc != 0:
            self._h = None
            _check(rc, None)
        self.N = pos.shape[0]
        self.lmax = lmax
        self.nmax = 2 * lmax * (lmax + 2)
        self.k = 2 * np.pi * n0 / wavelength
        self.options = opt

    def set_solve_options(self, **kw):
        """Change solver settings (precision, tol, inner_tol, restart, maxiter,
        max_refinements, verbose, solver, target_Nj, mem_cap_bytes, autotune,
        translation, deterministic)
        for the next solves, keeping geometry, incident field and
        preconditioner (celes_set_solve_options)."""
        opt = Options()
        C.memmove(C.byref(opt), C.byref(self.options), C.sizeof(Options))
        for k, v in kw.items():
            if not hasattr(opt, k):
                raise KeyError(k)
            setattr(opt, k, v)
        _check(lib().celes_set_solve_options(self._h, C.byref(opt)), self._h)
        self.options = opt

    def close(self):
        if getattr(self, "_h", None):
            lib().celes_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- incident field -------------------------------------------------
    def set_plane_waves(self, beta, alpha, pol, E0=None):
        beta = np.ascontiguousarray(np.atleast_1d(beta), dtype=np.float64)
        alpha = np.ascontiguousarray(np.atleast_1d(alpha), dtype=np.float64)
        pol = np.ascontiguousarray(np.atleast_1d(pol), dtype=np.int32)
        K = beta.size
        e = None
        if E0 is not None:
            z = np.broadcast_to(np.asarray(E0, dtype=np.complex128), (K,))
            e = np.ascontiguousarray(np.stack([z.real, z.imag], -1))
        _check(lib().celes_set_plane_waves(self._h, K, _dptr(beta), _dptr(alpha),
                                           pol.ctypes.data_as(C.POINTER(C.c_int)),
                                           _dptr(e) if e is not None else None), self._h)

    def set_gaussian_beam(self, waist, focus, alpha_G, E0=1.0, n_beta=512):
        f = np.ascontiguousarray(focus, dtype=np.float64)
        _check(lib().celes_set_gaussian_beam(self._h, float(waist), _dptr(f), float(alpha_G), float(np.real(E0)),
                                             float(np.imag(E0)), int(n_beta)), self._h)

    @property
    def num_rhs(self):
        return lib().celes_num_rhs(self._h)

    def incident(self):
        K = self.num_rhs
        out = np.zeros((K, self.N, self.nmax), dtype=np.complex128)
        _check(lib().celes_get_incident(self._h, _dptr(out.view(np.float64))), self._h)
        return out

    # ---- solve ------------------------------------------------------------
    def build_preconditioner(self, cuboid_edge=CELES_CUBOID_AUTO):
        """Block-diagonal preconditioner with cubes of edge cuboid_edge (0:
        remove it; CELES_CUBOID_AUTO: the budgeted edge from the options'
        target_Nj and mem_cap_bytes).  Returns (edge, cuboids, bytes)."""
        _check(lib().celes_build_preconditioner(self._h, float(cuboid_edge)), self._h)
        return self.preconditioner_info()

    def preconditioner_info(self):
        e, nb, by = C.c_double(), C.c_int64(), C.c_double()
        _check(lib().celes_preconditioner_info(self._h, C.byref(e), C.byref(nb), C.byref(by)), self._h)
        return e.value, nb.value, by.value

    def solve(self, x0=None, check=True):
        K = self.num_rhs
        b = np.zeros((K, self.N, self.nmax), dtype=np.complex128)
        info = SolveInfo()
        x = None
        if x0 is not None:
            x = np.ascontiguousarray(np.broadcast_to(x0, b.shape), dtype=np.complex128)
        rc = lib().celes_solve(self._h, _dptr(x.view(np.float64)) if x is not None else None,
                               _dptr(b.view(np.float64)), C.byref(info))
        if check and rc not in (0,):
            _check(rc, self._h)
        return b, {f: getattr(info, f) for f, _ in SolveInfo._fields_}

    def subsystem_guess(self, idx, cuboid_edge=0.0, check=True):
        """Initial guess [K][N][nmax] from solving the sub-ensemble idx alone
        (celes_subsystem_guess); returns (x0, info of the sub-solve)."""
        ix = np.ascontiguousarray(np.atleast_1d(idx), dtype=np.int64)
        x0 = np.zeros((self.num_rhs, self.N, self.nmax), dtype=np.complex128)
        info = SolveInfo()
        rc = lib().celes_subsystem_guess(self._h, ix.size, ix.ctypes.data_as(C.POINTER(C.c_int64)),
                                         float(cuboid_edge), _dptr(x0.view(np.float64)), C.byref(info))
        if check and rc != 0:
            _check(rc, self._h)
        return x0, {f: getattr(info, f) for f, _ in SolveInfo._fields_}

    def apply_W(self, x, y, precision=CELES_FP64, stream=None, K=1):
        """y = W x on device buffers (torch tensors or raw pointers)."""
        xp = x.data_ptr() if hasattr(x, "data_ptr") else int(x)
        yp = y.data_ptr() if hasattr(y, "data_ptr") else int(y)
        _check(lib().celes_apply_W(self._h, precision, K, C.c_void_p(xp), C.c_void_p(yp), _stream_ptr(stream)),
               self._h)

    def apply_W_noalloc(self, x, y, precision=CELES_FP64, stream=None, K=1):
        """y = W x with the library's fixed scratch array (celes_apply_W_noalloc)."""
        xp = x.data_ptr() if hasattr(x, "data_ptr") else int(x)
        yp = y.data_ptr() if hasattr(y, "data_ptr") else int(y)
        _check(lib().celes_apply_W_noalloc(self._h, precision, K, C.c_void_p(xp), C.c_void_p(yp),
                                           _stream_ptr(stream)), self._h)

    def apply_M(self, x, y, precision=CELES_FP64, stream=None, K=1):
        xp = x.data_ptr() if hasattr(x, "data_ptr") else int(x)
        yp = y.data_ptr() if hasattr(y, "data_ptr") else int(y)
        _check(lib().celes_apply_M(self._h, precision, K, C.c_void_p(xp), C.c_void_p(yp), _stream_ptr(stream)),
               self._h)

    def apply_preconditioner(self, x, y, precision=CELES_FP64, stream=None, K=1):
        """y = P^{-1} x (block-diagonal preconditioner) for K right-hand sides
        on device buffers."""
        xp = x.data_ptr() if hasattr(x, "data_ptr") else int(x)
        yp = y.data_ptr() if hasattr(y, "data_ptr") else int(y)
        _check(lib().celes_apply_preconditioner(self._h, precision, int(K), C.c_void_p(xp), C.c_void_p(yp),
                                                _stream_ptr(stream)), self._h)

    # ---- observables ------------------------------------------------------
    def cross_sections(self):
        K = self.num_rhs
        ce, cs, ca = np.zeros(K), np.zeros(K), np.zeros(K)
        _check(lib().celes_cross_sections(self._h, _dptr(ce), _dptr(cs), _dptr(ca)), self._h)
        return ce, cs, ca

    def power_flux(self, n_beta=0, n_alpha=0):
        """Per right-hand side (P_inc / I_0, R, T, A) of the last solution under
        a Gaussian beam; R + T + A = 1."""
        out = np.zeros((self.num_rhs, 4))
        _check(lib().celes_power_flux(self._h, int(n_beta), int(n_alpha), _dptr(out)), self._h)
        return out

    def far_field(self, theta, phi):
        th = np.ascontiguousarray(np.atleast_1d(theta), dtype=np.float64)
        ph = np.ascontiguousarray(np.atleast_1d(phi), dtype=np.float64)
        out = np.zeros((self.num_rhs, th.size, 3), dtype=np.complex128)
        _check(lib().celes_far_field(self._h, th.size, _dptr(th), _dptr(ph), _dptr(out.view(np.float64))), self._h)
        return out

    def near_field(self, points, add_incident=True):
        p = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
        out = np.zeros((self.num_rhs, p.shape[0], 3), dtype=np.complex128)
        _check(lib().celes_near_field(self._h, p.shape[0], _dptr(p), int(bool(add_incident)),
                                      _dptr(out.view(np.float64))), self._h)
        return out

    def solution(self):
        out = np.zeros((self.num_rhs, self.N, self.nmax), dtype=np.complex128)
        _check(lib().celes_get_solution(self._h, _dptr(out.view(np.float64))), self._h)
        return out

    def kernel_timing(self, enable):
        """Start (enable=True) or stop kernel timing; stopping returns the
        average coupling-kernel duration in ms and the launch count."""
        ms, n = C.c_double(0.0), C.c_int(0)
        _check(lib().celes_kernel_timing(self._h, 1 if enable else 0, C.byref(ms), C.byref(n)), self._h)
        return None if enable else (ms.value, n.value)

    def lut_info(self):
        lo, dr, n = C.c_double(), C.c_double(), C.c_int64()
        _check(lib().celes_lut_info(self._h, C.byref(lo), C.byref(dr), C.byref(n)), self._h)
        return lo.value, dr.value, n.value


def _bcheck(rc, b=None):
    if rc != 0:
        msg = lib().celes_batch_last_error(b)
        raise CelesError(rc, msg.decode() if msg else "")


class Batch:
    """Independent problems solved together (celes_batch_*): one persistent
    mat-vec launch per Arnoldi step over all problems and right-hand sides."""

    def __init__(self, problems, options=None, **kw):
        self.problems = list(problems)
        arr = (C.c_void_p * len(self.problems))(*[p._h.value for p in self.problems])
        opt = options if options is not None else default_options(**kw)
        self._b = C.c_void_p()
        rc = lib().celes_batch_create(C.byref(self._b), len(self.problems), arr, C.byref(opt))
        if rc != 0:
            self._b = None
            _bcheck(rc, None)
        self.options = opt

    @property
    def num_systems(self):
        return lib().celes_batch_num_systems(self._b)

    def close(self):
        if getattr(self, "_b", None):
            lib().celes_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply_M(self, x, y, precision=CELES_FP64, stream=None):
        xp = x.data_ptr() if hasattr(x, "data_ptr") else int(x)
        yp = y.data_ptr() if hasattr(y, "data_ptr") else int(y)
        _bcheck(lib().celes_batch_apply_M(self._b, precision, C.c_void_p(xp), C.c_void_p(yp), _stream_ptr(stream)),
                self._b)

    def autotune(self, precision=CELES_MIXED):
        ms, ch, kb = C.c_double(), C.c_int(), C.c_int()
        _bcheck(lib().celes_batch_autotune(self._b, precision, C.byref(ms), C.byref(ch), C.byref(kb)), self._b)
        return {"ms": ms.value, "chunk_len": ch.value, "kb": kb.value}

    def solve(self, check=True):
        n = self.num_systems
        infos = (SolveInfo * n)()
        summ = SolveInfo()
        rc = lib().celes_batch_solve(self._b, infos, C.byref(summ))
        if check and rc != 0:
            _bcheck(rc, self._b)
        per = [{f: getattr(i, f) for f, _ in SolveInfo._fields_} for i in infos]
        return per, {f: getattr(summ, f) for f, _ in SolveInfo._fields_}


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Network:
    """Learned initial guess (celes_nn_*): 16-neighbour features, three
    hidden layers of 128, bf16 weights, FP32 accumulation, trained on the
    solver's own output."""

    def __init__(self, lmax, seed=0):
        self._n = C.c_void_p()
        rc = lib().celes_nn_create(C.byref(self._n), int(lmax), C.c_uint64(seed))
        if rc != 0:
            raise CelesError(rc, "celes_nn_create failed")
        a = [C.c_int() for _ in range(5)]
        npar = C.c_int64()
        lib().celes_nn_dims(self._n, *[C.byref(x) for x in a], C.byref(npar))
        self.in_dim, self.in_pad, self.hidden, self.out_dim, self.out_pad = [x.value for x in a]
        self.nparam = npar.value
        self.lmax = lmax

    def _check(self, rc):
        if rc != 0:
            msg = lib().celes_nn_last_error(self._n)
            raise CelesError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_n", None):
            lib().celes_nn_destroy(self._n)
            self._n = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        p = np.zeros(self.nparam, dtype=np.float32)
        self._check(lib().celes_nn_get_params(self._n, _fptr(p)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparam
        self._check(lib().celes_nn_set_params(self._n, _fptr(p)))

    def features(self, problem, targets=True):
        X = np.zeros((problem.N, self.in_pad), dtype=np.float32)
        Y = np.zeros((problem.N, self.out_pad), dtype=np.float32) if targets else None
        self._check(lib().celes_nn_features(self._n, problem._h, _fptr(X), _fptr(Y) if Y is not None else None))
        return X, Y

    def loss_grad(self, X, Y):
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        g = np.zeros(self.nparam, dtype=np.float32)
        loss = C.c_double()
        self._check(lib().celes_nn_loss_grad(self._n, X.shape[0], _fptr(X), _fptr(Y), C.byref(loss), _fptr(g)))
        return loss.value, g

    def forward(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        Z = np.zeros((X.shape[0], self.out_pad), dtype=np.float32)
        self._check(lib().celes_nn_forward(self._n, X.shape[0], _fptr(X), _fptr(Z)))
        return Z

    def add_training_problem(self, problem):
        self._check(lib().celes_nn_add_training_problem(self._n, problem._h))

    def train(self, epochs, batch=1024, lr=1e-3, seed=0):
        loss = C.c_double()
        self._check(lib().celes_nn_train(self._n, int(epochs), int(batch), float(lr), C.c_uint64(seed),
                                         C.byref(loss)))
        return loss.value

    def predict(self, problem):
        x0 = np.zeros((problem.N, problem.nmax), dtype=np.complex128)
        self._check(lib().celes_nn_predict(self._n, problem._h, _dptr(x0.view(np.float64))))
        return x0
