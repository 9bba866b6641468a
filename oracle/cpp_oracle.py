"""ctypes front of the C++ FP64 oracle (oracle/wfq_oracle.cpp) -- TEST INFRASTRUCTURE ONLY.

`CppProblem` offers the interface of the Python oracle's `Problem` (apply_T, z, rhs, apply, residual,
residual_rows, solve_lu, solve_gmres, solve_qmr, L, sample_T) so that the same pins run against both
oracles. The library is built by oracle/build_oracle.py (and by the package build entry point); it is
loaded as built, and built here only if it is missing.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
import scipy.sparse

from .build_oracle import LIB, build

_DP = C.POINTER(C.c_double)
_I64P = C.POINTER(C.c_int64)
_IP = C.POINTER(C.c_int)
_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = C.CDLL(LIB)
        sig = {
            "orc_create": (C.c_void_p, [C.c_int64, _DP, _DP, _DP, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_double, C.c_int]),
            "orc_destroy": (None, [C.c_void_p]),
            "orc_threads": (C.c_int, []),
            "orc_nnz": (C.c_int64, [C.c_void_p]),
            "orc_export_L": (C.c_int, [C.c_void_p, _I64P, _I64P, _DP]),
            "orc_sample_T": (None, [C.c_void_p, C.c_int64, _I64P, _I64P, _DP]),
            "orc_apply_T": (None, [C.c_void_p, C.c_int, _DP, _DP]),
            "orc_apply_T_rows": (None, [C.c_void_p, C.c_int64, _I64P, C.c_int, _DP, _DP]),
            "orc_apply": (C.c_int, [C.c_void_p, C.c_double, C.c_double, _DP, _DP, _DP, _DP]),
            "orc_shift": (None, [C.c_void_p, C.c_double, _DP, _DP]),
            "orc_rhs": (C.c_int, [C.c_void_p, _DP, C.c_double, _DP]),
            "orc_solve_lu": (C.c_int, [C.c_void_p, C.c_double, _DP, C.c_double, _DP, _DP]),
            "orc_residual": (C.c_double, [C.c_void_p, C.c_double, _DP, C.c_double, _DP, _DP]),
            "orc_residual_rows": (None, [C.c_void_p, C.c_double, _DP, C.c_double, _DP, _DP, C.c_int64, _I64P,
                                         _DP, _DP]),
            "orc_gmres": (C.c_int, [C.c_void_p, C.c_double, _DP, C.c_double, C.c_int, C.c_double, C.c_int, _DP,
                                    _DP, _DP, _DP, _IP, _DP]),
            "orc_qmr": (C.c_int, [C.c_void_p, C.c_double, _DP, C.c_double, C.c_double, C.c_int, C.c_double, _DP,
                                  _DP, _IP, _DP]),
            "orc_polarisability": (None, [C.c_void_p, _DP, _DP, C.c_double, _DP, _DP]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def threads() -> int:
    return int(load().orc_threads())


def _dp(a):
    return a.ctypes.data_as(_DP) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class CppProblem:
    """One structure in the C++ oracle. dense_T stores T (n^2 doubles); build_L builds the whole L
    (all-pairs search); without it only residual_rows and T products are available."""

    def __init__(self, xyz_A, params, dense_T=True, build_L=True, species=None):
        from .wfq_oracle import atom_parameters, material_weight
        xyz = _f64(xyz_A).reshape(-1, 3)
        self.n = xyz.shape[0]
        self.xyz = xyz / 0.529177210903
        eta, r0 = atom_parameters(params, self.n, species)
        self._keep = (xyz, eta, r0)
        mode = (1 if dense_T else 0) | (2 if build_L else 0)
        self.ptr = load().orc_create(self.n, _dp(xyz), _dp(eta), _dp(r0), float(params["fermi_d"]),
                                     float(params["fermi_s"]), float(params["cutoff_eps"]), material_weight(params),
                                     float(params["tau"]), mode)
        if not self.ptr:
            raise ValueError("C++ oracle rejected the structure")
        self._L = None

    def __del__(self):
        try:
            if self.ptr:
                load().orc_destroy(self.ptr)
                self.ptr = None
        except Exception:
            pass

    @property
    def L(self):
        if self._L is None:
            nnz = int(load().orc_nnz(self.ptr))
            if nnz < 0:
                raise ValueError("L was not built")
            r, c = np.zeros(nnz, np.int64), np.zeros(nnz, np.int64)
            v = np.zeros(nnz)
            load().orc_export_L(self.ptr, r.ctypes.data_as(_I64P), c.ctypes.data_as(_I64P), _dp(v))
            self._L = scipy.sparse.csr_matrix((v, (r, c)), shape=(self.n, self.n))
        return self._L

    def sample_T(self, i, j):
        i = np.ascontiguousarray(i, dtype=np.int64)
        j = np.ascontiguousarray(j, dtype=np.int64)
        out = np.zeros(len(i))
        load().orc_sample_T(self.ptr, len(i), i.ctypes.data_as(_I64P), j.ctypes.data_as(_I64P), _dp(out))
        return out

    def apply_T(self, x):
        x = np.asarray(x)
        cplx = np.iscomplexobj(x)
        flat = x.reshape(self.n, -1)
        parts = [flat.real, flat.imag] if cplx else [flat]
        outs = []
        for part in parts:
            X = _f64(part.T)
            Y = np.zeros_like(X)
            load().orc_apply_T(self.ptr, X.shape[0], _dp(X), _dp(Y))
            outs.append(Y.T)
        y = outs[0] + 1j * outs[1] if cplx else outs[0]
        return y.reshape(x.shape)

    def apply_T_rows(self, rows, X):
        """(T X)[rows] for real X (n, ncol), from pairwise elements."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        Xc = _f64(np.asarray(X, dtype=np.float64).reshape(self.n, -1).T)
        Y = np.zeros((Xc.shape[0], len(rows)))
        load().orc_apply_T_rows(self.ptr, len(rows), rows.ctypes.data_as(_I64P), Xc.shape[0], _dp(Xc), _dp(Y))
        return Y.T

    def z(self, omega_eV):
        zr, zi = C.c_double(), C.c_double()
        load().orc_shift(self.ptr, float(omega_eV), C.byref(zr), C.byref(zi))
        return complex(zr.value, zi.value)

    def rhs(self, direction, E0=1.0):
        d = _f64(direction)
        b = np.zeros(self.n)
        if load().orc_rhs(self.ptr, _dp(d), float(E0), _dp(b)) != 0:
            raise ValueError("L was not built")
        return b

    def apply(self, z):
        def f(x):
            x = np.asarray(x, dtype=np.complex128)
            xr, xi = _f64(x.real), _f64(x.imag)
            yr, yi = np.zeros(self.n), np.zeros(self.n)
            load().orc_apply(self.ptr, z.real, z.imag, _dp(xr), _dp(xi), _dp(yr), _dp(yi))
            return yr + 1j * yi
        return f

    def residual(self, omega_eV, direction, q, E0=1.0):
        q = np.asarray(q, dtype=np.complex128)
        d = _f64(direction)
        return float(load().orc_residual(self.ptr, float(omega_eV), _dp(d), float(E0), _dp(_f64(q.real)),
                                         _dp(_f64(q.imag))))

    def residual_rows(self, omega_eV, direction, q, rows, E0=1.0):
        q = np.asarray(q, dtype=np.complex128)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        d = _f64(direction)
        orr, ori = np.zeros(len(rows)), np.zeros(len(rows))
        load().orc_residual_rows(self.ptr, float(omega_eV), _dp(d), float(E0), _dp(_f64(q.real)), _dp(_f64(q.imag)),
                                 len(rows), rows.ctypes.data_as(_I64P), _dp(orr), _dp(ori))
        return orr + 1j * ori

    def solve_lu(self, omega_eV, direction, E0=1.0):
        d = _f64(direction)
        qr, qi = np.zeros(self.n), np.zeros(self.n)
        rc = load().orc_solve_lu(self.ptr, float(omega_eV), _dp(d), float(E0), _dp(qr), _dp(qi))
        if rc != 0:
            raise ValueError(f"LU failed ({rc})")
        return qr + 1j * qi

    def solve_gmres(self, omega_eV, direction, restart, tol, maxiter=100000, E0=1.0, x0=None):
        d = _f64(direction)
        qr, qi = np.zeros(self.n), np.zeros(self.n)
        info = (C.c_int * 2)()
        rel = C.c_double()
        x0r = _f64(np.real(x0)) if x0 is not None else None
        x0i = _f64(np.imag(x0)) if x0 is not None else None
        rc = load().orc_gmres(self.ptr, float(omega_eV), _dp(d), float(E0), int(restart), float(tol), int(maxiter),
                              _dp(x0r), _dp(x0i), _dp(qr), _dp(qi), info, C.byref(rel))
        if rc != 0:
            raise ValueError("GMRES failed")
        return qr + 1j * qi, dict(iters=info[0], cycles=info[1], relres=rel.value)

    def solve_qmr(self, omega_eV, direction, tol, maxiter=100000, E0=1.0, breakdown=1e-14):
        d = _f64(direction)
        qr, qi = np.zeros(self.n), np.zeros(self.n)
        info = (C.c_int * 2)()
        rel = C.c_double()
        rc = load().orc_qmr(self.ptr, float(omega_eV), _dp(d), float(E0), float(tol), int(maxiter),
                            float(breakdown), _dp(qr), _dp(qi), info, C.byref(rel))
        if rc != 0:
            raise ValueError("QMR failed")
        return qr + 1j * qi, dict(iters=info[0], breakdown=bool(info[1]), relres=rel.value)

    def polarisability(self, Q, E0=1.0):
        """alpha[l, k] for the columns k of Q (N, n_dir)."""
        Q = np.asarray(Q, dtype=np.complex128).reshape(self.n, -1)
        out = np.zeros((3, Q.shape[1]), dtype=np.complex128)
        for k in range(Q.shape[1]):
            ar, ai = np.zeros(3), np.zeros(3)
            load().orc_polarisability(self.ptr, _dp(_f64(Q[:, k].real)), _dp(_f64(Q[:, k].imag)), float(E0),
                                      _dp(ar), _dp(ai))
            out[:, k] = ar + 1j * ai
        return out
