"""Test infrastructure: reference (oracle) code.  Only ``tests/``, the smoke
check and the benchmark's CPU-baseline leg may import it.

Full-CI oracle (O-FCI): the Hamiltonian of Sec. II.A (Eq. ``Hamiltonian``)
on the determinant basis of a fixed ``(n_up, n_dn)`` sector, the space in
which the full-CI tensor of Eq. ``fulltensor`` lives.  The determinant
action itself is the plain C in ``fci.c``.

Pinned by (``tests/test_oracle_fci.py``): the V=0 closed form (sum of
orbital energies), the Hubbard dimer closed form, and the spinless 4x4
torus energies the paper prints (Sec. III.A).
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_fci.so")
_lib = None


def build_lib(force=False):
    """Compile ``fci.c`` with gcc into ``oracle/_fci.so``."""
    src = os.path.join(_HERE, "fci.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build_lib()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        up = ctypes.POINTER(ctypes.c_uint64)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib.fci_apply_det.argtypes = [ctypes.c_int, dp, dp, up, up, dp, ctypes.c_int64]
        lib.fci_apply_det.restype = ctypes.c_int64
        lib.fci_row_dot.argtypes = [ctypes.c_int, dp, dp, up, ctypes.c_int64, up, dp]
        lib.fci_row_dot.restype = ctypes.c_double
        lib.fci_build_coo.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int64, up, ip, ip, dp, ctypes.c_int64]
        lib.fci_build_coo.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


# ---------------------------------------------------------------------------
# determinant strings: mode m = 2*i + sigma (sigma 0=up, 1=down)
# ---------------------------------------------------------------------------
def det_from_occ(up_orbs, dn_orbs):
    """Two-word (lo, hi) bit string of a determinant."""
    v = 0
    for i in up_orbs:
        v |= 1 << (2 * i)
    for i in dn_orbs:
        v |= 1 << (2 * i + 1)
    return np.array([v & 0xFFFFFFFFFFFFFFFF, v >> 64], dtype=np.uint64)


def det_to_int(d):
    return int(d[0]) | (int(d[1]) << 64)


def sector_dets(n_orb, n_up, n_dn):
    """All determinants of the sector, sorted ascending as 128-bit integers.
    Returns an (n, 2) uint64 array of (lo, hi) words."""
    ups = [sum(1 << (2 * i) for i in c) for c in itertools.combinations(range(n_orb), n_up)]
    dns = [sum(1 << (2 * i + 1) for i in c) for c in itertools.combinations(range(n_orb), n_dn)]
    vals = sorted(u | d for u in ups for d in dns)
    out = np.empty((len(vals), 2), dtype=np.uint64)
    for k, v in enumerate(vals):
        out[k, 0] = v & 0xFFFFFFFFFFFFFFFF
        out[k, 1] = v >> 64
    return out


def hamiltonian(h, V, n_up, n_dn, basis=None):
    """Sparse H on the sorted sector basis (CSR, duplicates summed)."""
    lib = _load()
    n = h.shape[0]
    h = np.ascontiguousarray(h, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    if basis is None:
        basis = sector_dets(n, n_up, n_dn)
    basis = np.ascontiguousarray(basis, dtype=np.uint64)
    nb = basis.shape[0]
    cnt = lib.fci_build_coo(n, _p(h, ctypes.c_double), _p(V, ctypes.c_double), nb,
                            _p(basis, ctypes.c_uint64), None, None, None, 0)
    rows = np.empty(cnt, dtype=np.int64)
    cols = np.empty(cnt, dtype=np.int64)
    vals = np.empty(cnt, dtype=np.float64)
    lib.fci_build_coo(n, _p(h, ctypes.c_double), _p(V, ctypes.c_double), nb,
                      _p(basis, ctypes.c_uint64), _p(rows, ctypes.c_int64),
                      _p(cols, ctypes.c_int64), _p(vals, ctypes.c_double), cnt)
    return sp.coo_matrix((vals, (rows, cols)), shape=(nb, nb)).tocsr(), basis


def lowest(h, V, n_up, n_dn, k=1):
    """Lowest k eigenvalues (ascending) of H in the sector."""
    H, _ = hamiltonian(h, V, n_up, n_dn)
    if H.shape[0] <= 3000:
        w = np.linalg.eigvalsh(H.toarray())
        return w[:k]
    w = spla.eigsh(H, k=k, which="SA", tol=1e-13, return_eigenvectors=False)
    return np.sort(w)


def apply_det(h, V, det):
    """Terms of H|det> as (list of 128-bit ints, values), unsummed."""
    lib = _load()
    n = h.shape[0]
    h = np.ascontiguousarray(h, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    det = np.ascontiguousarray(det, dtype=np.uint64)
    cnt = lib.fci_apply_det(n, _p(h, ctypes.c_double), _p(V, ctypes.c_double),
                            _p(det, ctypes.c_uint64), None, None, 0)
    od = np.empty((cnt, 2), dtype=np.uint64)
    ov = np.empty(cnt, dtype=np.float64)
    lib.fci_apply_det(n, _p(h, ctypes.c_double), _p(V, ctypes.c_double),
                      _p(det, ctypes.c_uint64), _p(od, ctypes.c_uint64),
                      _p(ov, ctypes.c_double), cnt)
    return od, ov


def row_dot(h, V, det, basis, x):
    """sum_j <basis_j|H|det> x_j for a sorted basis (= (H x)[det])."""
    lib = _load()
    n = h.shape[0]
    h = np.ascontiguousarray(h, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    det = np.ascontiguousarray(det, dtype=np.uint64)
    basis = np.ascontiguousarray(basis, dtype=np.uint64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib.fci_row_dot(n, _p(h, ctypes.c_double), _p(V, ctypes.c_double),
                           _p(det, ctypes.c_uint64), basis.shape[0],
                           _p(basis, ctypes.c_uint64), _p(x, ctypes.c_double))
