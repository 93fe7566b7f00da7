"""Python binding of the HIP library ``libheff.so`` (C ABI in include/heff.h).

Argument marshalling only: every arithmetic step of the two-site H_eff
path runs in the library's HIP kernels.  PyTorch provides device memory and
the current stream.  Importing this module fails loudly when the built
library is missing.
"""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libheff.so")

FP64, FP32, BF16X3 = 0, 1, 2
KEEP_ENV = 1 << 8  # build flag: keep the environment of later sweep steps
PREC_NAMES = {FP64: "fp64", FP32: "fp32", BF16X3: "bf16x3"}

# operator kinds of heff_debug_op
K_H, K_C, K_A, K_B, K_T, K_D, K_DD, K_BB, K_S = range(9)

if not os.path.exists(LIB_PATH):
    raise ImportError("libheff.so is not built (run __graft_entry__.build()): " + LIB_PATH)
# PyTorch is loaded before the library: its bundled HIP runtime then serves
# the library's libamdhip64.so.7 dependency too.  Loaded the other way
# round, the library binds the system runtime and PyTorch later loads its
# own copy under another file name: two HIP runtimes in one process, and
# the library's context creation fails on the GPU.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)


class _Bond(ctypes.Structure):
    _fields_ = [("n_sect", ctypes.c_int32), ("nup", ctypes.POINTER(ctypes.c_int32)),
                ("ndn", ctypes.POINTER(ctypes.c_int32)), ("dim", ctypes.POINTER(ctypes.c_int32))]


class _Problem(ctypes.Structure):
    _fields_ = [("n_orb", ctypes.c_int32), ("n_up", ctypes.c_int32), ("n_dn", ctypes.c_int32),
                ("h", ctypes.POINTER(ctypes.c_double)), ("V", ctypes.POINTER(ctypes.c_double)),
                ("left", ctypes.POINTER(_Bond)), ("right", ctypes.POINTER(_Bond)),
                ("iso_left", ctypes.POINTER(ctypes.POINTER(ctypes.c_double))),
                ("iso_right", ctypes.POINTER(ctypes.POINTER(ctypes.c_double)))]


_vp = ctypes.c_void_p
_i = ctypes.c_int

_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)
_F64P = ctypes.POINTER(ctypes.c_double)


class _Su2Block(ctypes.Structure):
    _fields_ = [("n_sect", ctypes.c_int32), ("n", _I32P), ("two_s", _I32P), ("dim", _I32P),
                ("n_ops", ctypes.c_int32), ("two_k", _I32P), ("dn", _I32P),
                ("n_blk", ctypes.c_int64), ("blk_op", _I32P), ("blk_out", _I32P), ("blk_in", _I32P),
                ("blk_off", _I64P), ("data", _F64P), ("data_len", ctypes.c_int64)]


class _Su2Problem(ctypes.Structure):
    _fields_ = [("left", _Su2Block), ("right", _Su2Block), ("n_terms", ctypes.c_int32),
                ("term_l", _I32P), ("term_site_k", _I32P), ("term_site_k1", _I32P), ("term_r", _I32P),
                ("term_two_s", _I32P), ("term_coef", _F64P), ("n_tot", ctypes.c_int32), ("two_s_tot", ctypes.c_int32)]



# heff_alloc: device memory provider callbacks
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class _Alloc(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


# user key -> (alloc(nbytes) -> int address or 0, free(address)); keys start
# at 1 (a zero `user` arrives as None).  Entries live as long as the module:
# library objects free through them after their context is gone.
_PROVIDERS = {}


def _alloc_cb(nbytes, user):
    try:
        return _PROVIDERS[user][0](int(nbytes)) or None
    except Exception:  # any failure is a refusal: the library reports HEFF_ENOMEM
        return None


def _free_cb(ptr, user):
    try:
        _PROVIDERS[user][1](int(ptr))
    except Exception:
        pass


_ALLOC_CB = _ALLOC_FN(_alloc_cb)
_FREE_CB = _FREE_FN(_free_cb)


def _torch_provider(device, stream):
    """PyTorch's caching allocator on (device, stream): the library's device
    memory is then owned by torch."""
    import torch
    handle = stream.cuda_stream

    def alloc(n):
        return torch.cuda.caching_allocator_alloc(max(n, 1), device, handle)

    def free(ptr):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, free


def _register_provider(fns):
    key = len(_PROVIDERS) + 1
    _PROVIDERS[key] = fns
    return _Alloc(_ALLOC_CB, _FREE_CB, key)


_lib.heff_create.argtypes = [ctypes.POINTER(_vp), _i, _vp, ctypes.POINTER(_Alloc)]
_lib.heff_destroy.argtypes = [_vp]
_lib.heff_last_error.argtypes = [_vp]
_lib.heff_last_error.restype = ctypes.c_char_p
_lib.heff_build_blocks.argtypes = [_vp, ctypes.POINTER(_Problem), ctypes.c_uint32, ctypes.POINTER(_vp)]
_lib.heff_validate_problem.argtypes = [ctypes.POINTER(_Problem), ctypes.c_char_p, ctypes.c_int32]
_lib.heff_blocks_free.argtypes = [_vp]
_lib.heff_psi_layout.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
                                 ctypes.POINTER(ctypes.POINTER(ctypes.c_int64))]
_lib.heff_task_stats.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)]
_lib.heff_apply.argtypes = [_vp, _vp, _i, _vp, _vp]
_lib.heff_diag.argtypes = [_vp, _vp, _vp]
_lib.heff_dav_create.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.c_double, _vp, ctypes.POINTER(_vp)]
_lib.heff_davidson_step.argtypes = [_vp, _vp, _i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
_lib.heff_dav_ritz.argtypes = [_vp, _vp, _vp]
_lib.heff_dav_free.argtypes = [_vp]
_lib.heff_timing.argtypes = [_vp, _i]
_lib.heff_timing_read.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
_lib.heff_task_stats_variant.argtypes = [_vp, _i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
_lib.heff_blocks_shard.argtypes = [_vp, _vp, _i, _i, ctypes.POINTER(ctypes.c_double)]
_lib.heff_task_stats_issued.argtypes = [_vp, _i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64)]
_lib.heff_truncate.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.POINTER(_vp)]
_lib.heff_trunc_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
_lib.heff_trunc_get.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _vp]
_lib.heff_trunc_free.argtypes = [_vp]
_lib.heff_sweep_right.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(_vp), ctypes.POINTER(_vp)]
_lib.heff_start_vector.argtypes = [_vp, ctypes.POINTER(ctypes.POINTER(ctypes.c_double))]
_lib.heff_rotate_pair.argtypes = [_vp, _vp, ctypes.c_double, _vp, _vp]
_lib.heff_pair_entropy.argtypes = [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
_lib.heff_optimize_pair.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
_lib.heff_rotate_integrals.argtypes = [ctypes.c_int32, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                       _vp, _vp]
_lib.heff_batch_layout.argtypes = [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int64)]
_lib.heff_batch_create.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int32, _vp, _vp, ctypes.POINTER(_vp)]
_lib.heff_batch_set_grid.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32)]
_lib.heff_energy.argtypes = [_vp, _vp, _i, _vp, ctypes.POINTER(ctypes.c_double)]
_lib.heff_energy_noalloc.argtypes = [_vp, _vp, _i, _vp, ctypes.POINTER(ctypes.c_double)]
_lib.heff_energy_backward.argtypes = [_vp, _vp, _i, _vp, ctypes.c_double, _vp, _vp, _vp]
_lib.heff_op_arena.argtypes = [_vp, _i, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_int64)]
_lib.heff_kappa_gradient.argtypes = [_vp, ctypes.POINTER(_Problem), _vp, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
_lib.heff_set_fp64_kernel.argtypes = [_vp, ctypes.c_int32]
_lib.heff_integral_gradient.argtypes = [_vp, ctypes.POINTER(_Problem), _vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]
_lib.heff_batch_io.argtypes = [_vp, ctypes.POINTER(ctypes.POINTER(ctypes.c_int64)), ctypes.POINTER(ctypes.c_int64)]
_lib.heff_batch_stats.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int64)]
_lib.heff_batch_apply.argtypes = [_vp, _vp, _i]
_lib.heff_batch_free.argtypes = [_vp]
_lib.heff_debug_op.argtypes = [_vp, _i, _i, _i, _i, ctypes.POINTER(ctypes.c_double), ctypes.c_int64]
_lib.heff_debug_op.restype = ctypes.c_int64
_lib.heff_su2_create.argtypes = [_vp, ctypes.POINTER(_Su2Problem), ctypes.c_uint32, ctypes.POINTER(_vp)]
_lib.heff_su2_layout.argtypes = [_vp, _I64P, _I32P, ctypes.POINTER(_I32P), ctypes.POINTER(_I64P)]
_lib.heff_su2_stats.argtypes = [_vp, _I64P, _F64P, _F64P]
_lib.heff_su2_apply.argtypes = [_vp, _vp, _i, _vp, _vp]
_lib.heff_su2_free.argtypes = [_vp]
_lib.heff_su2_factor.argtypes = [_I32P, _F64P]

EXPORTED = ("heff_create", "heff_destroy", "heff_last_error", "heff_build_blocks", "heff_validate_problem",
            "heff_blocks_free",
            "heff_psi_layout", "heff_task_stats", "heff_apply", "heff_diag", "heff_dav_create",
            "heff_davidson_step", "heff_dav_ritz", "heff_dav_free", "heff_timing", "heff_timing_read",
            "heff_task_stats_variant", "heff_task_stats_issued", "heff_blocks_shard", "heff_energy", "heff_energy_backward",
            "heff_op_arena", "heff_energy_noalloc", "heff_kappa_gradient", "heff_integral_gradient", "heff_set_fp64_kernel", "heff_truncate", "heff_trunc_info", "heff_trunc_get", "heff_trunc_free",
            "heff_sweep_right", "heff_start_vector", "heff_rotate_pair", "heff_pair_entropy",
            "heff_optimize_pair", "heff_rotate_integrals",
            "heff_batch_layout", "heff_batch_create", "heff_batch_io", "heff_batch_set_grid", "heff_batch_stats",
            "heff_batch_apply", "heff_batch_free", "heff_su2_create", "heff_su2_layout", "heff_su2_stats",
            "heff_su2_apply", "heff_su2_free", "heff_su2_factor")
N_VARIANTS = 4
FP64_AUTO, FP64_STAGED, FP64_RING, FP64_RING_DWORD = 0, 1, 2, 3


class HeffError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("heff error %d: %s" % (code, msg))
        self.code = code


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())



HEFF_EINVAL, HEFF_ESECTOR, HEFF_ENOMEM, HEFF_EHIP, HEFF_ENOTSUP, HEFF_ENOCONV, HEFF_ESTATE = range(-1, -8, -1)


class Context:
    """Library context on a device, bound to torch's current stream.

    allocator: "torch" (default: every device buffer of the library comes
    from PyTorch's caching allocator on this stream), "hip" (the library's
    own hipMalloc / hipFree) or a pair of callables (alloc(nbytes) -> device
    address or 0, free(address))."""

    def __init__(self, device=0, stream=None, allocator="torch"):
        import torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        if allocator == "hip":
            prov = None
        elif allocator == "torch":
            prov = _register_provider(_torch_provider(device, stream))
        else:
            prov = _register_provider(tuple(allocator))
        self._prov = prov
        h = _vp()
        rc = _lib.heff_create(ctypes.byref(h), device, _vp(stream.cuda_stream),
                              ctypes.byref(prov) if prov is not None else None)
        if rc != 0:
            raise HeffError(rc, "heff_create failed")
        self._h = h

    def check(self, rc):
        if rc != 0:
            raise HeffError(rc, _lib.heff_last_error(self._h).decode())

    def timing(self, enable=True):
        """Enable/disable per-variant HIP-event timing of products (clears)."""
        self.check(_lib.heff_timing(self._h, 1 if enable else 0))

    def timing_read(self):
        """(ms[4], launches[4]) summed since the last clear; clears."""
        ms = (ctypes.c_double * N_VARIANTS)()
        n = (ctypes.c_int64 * N_VARIANTS)()
        self.check(_lib.heff_timing_read(self._h, ms, n))
        return list(ms), list(n)

    def set_fp64_kernel(self, mode):
        """Kernel family of the FP64 products: FP64_AUTO, FP64_STAGED or
        FP64_RING (bitwise identical results)."""
        self.check(_lib.heff_set_fp64_kernel(self._h, int(mode)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.heff_destroy(self._h)
            self._h = None

    def __del__(self, _fin=sys.is_finalizing):
        if _fin():  # the HIP runtime may already be gone
            return
        try:
            self.close()
        except Exception:
            pass


def _bond_array(tabs, keep):
    arr = (_Bond * len(tabs))()
    for i, t in enumerate(tabs):
        nu = np.array([q[0] for q in t], dtype=np.int32)
        nd = np.array([q[1] for q in t], dtype=np.int32)
        dm = np.array(list(t.values()), dtype=np.int32)
        keep += [nu, nd, dm]
        arr[i].n_sect = len(t)
        arr[i].nup = nu.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        arr[i].ndn = nd.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        arr[i].dim = dm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    return arr


def _marshal(p, keep, h=None, V=None):
    """heff_problem of a synth.Problem; arrays it points to go into `keep`."""
    from . import synth
    left = _bond_array(p.left, keep)
    right = _bond_array(p.right, keep)
    il = (ctypes.POINTER(ctypes.c_double) * max(1, len(p.iso_left)))()
    for i in range(len(p.iso_left)):
        a = np.ascontiguousarray(synth.iso_flat(p.left[i], p.left[i + 1], p.iso_left[i]))
        keep.append(a)
        il[i] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ir = (ctypes.POINTER(ctypes.c_double) * max(1, len(p.iso_right)))()
    for i in range(len(p.iso_right)):
        a = np.ascontiguousarray(synth.iso_flat(p.right[i], p.right[i + 1], p.iso_right[i]))
        keep.append(a)
        ir[i] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = np.ascontiguousarray(p.h if h is None else h, dtype=np.float64)
    V = np.ascontiguousarray(p.V if V is None else V, dtype=np.float64)
    keep += [h, V, il, ir]
    return _Problem(p.n_orb, p.n_up, p.n_dn, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    V.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), left, right, il, ir)


def validate_problem(problem, h=None, V=None):
    """Host-only checks of a problem (heff_validate_problem; no device):
    returns (code, message), code 0 when the problem is valid."""
    keep = []
    prob = _marshal(problem, keep, h, V)
    buf = ctypes.create_string_buffer(512)
    rc = _lib.heff_validate_problem(ctypes.byref(prob), buf, len(buf))
    return rc, buf.value.decode()


class _DeviceArray:
    """__cuda_array_interface__ of library-owned device memory, so that torch
    can view it without a copy."""

    def __init__(self, ptr, n, typestr, owner):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False), "version": 3}
        self._owner = owner


def _trunc_dict(ctx, h, device):
    """Contents of a truncation result: dict(sing, discarded, tab
    {(nu, nd): dim}, iso_flat (host copy of the isometry))."""
    import torch
    nk = ctypes.c_int32()
    disc = ctypes.c_double()
    ns = ctypes.c_int32()
    ln = ctypes.c_int64()
    _lib.heff_trunc_info(h, ctypes.byref(nk), ctypes.byref(disc), ctypes.byref(ns), ctypes.byref(ln))
    sing = np.empty(nk.value)
    nu = np.empty(ns.value, dtype=np.int32)
    nd = np.empty(ns.value, dtype=np.int32)
    dm = np.empty(ns.value, dtype=np.int32)
    iso = torch.empty(max(ln.value, 1), dtype=torch.float64, device=device)
    ctx.check(_lib.heff_trunc_get(ctx._h, h, sing.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  nu.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  nd.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  dm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(iso)))
    flat = iso[: ln.value].cpu().numpy()
    tab = {(int(a), int(b_)): int(d) for a, b_, d in zip(nu, nd, dm)}
    return dict(sing=sing, discarded=disc.value, tab=tab, iso_flat=flat)


class Blocks:
    """Renormalized operators + task table of one two-site problem."""

    def __init__(self, ctx: Context, problem, precs=(FP64,), keep_env=False, _handle=None):
        self.ctx = ctx
        self.precs = tuple(precs)
        if _handle is not None:  # blocks made by a sweep step
            out = _handle
        else:
            keep = []
            prob = _marshal(problem, keep)
            mask = KEEP_ENV if keep_env else 0
            for pr in precs:
                mask |= 1 << pr
            out = _vp()
            ctx.check(_lib.heff_build_blocks(ctx._h, ctypes.byref(prob), mask, ctypes.byref(out)))
        self._h = out
        n = ctypes.c_int64()
        nb = ctypes.c_int32()
        desc = ctypes.POINTER(ctypes.c_int32)()
        offs = ctypes.POINTER(ctypes.c_int64)()
        ctx.check(_lib.heff_psi_layout(out, ctypes.byref(n), ctypes.byref(nb), ctypes.byref(desc), ctypes.byref(offs)))
        self.n_elem = n.value
        self.blocks = [tuple(desc[6 * i + j] for j in range(6)) + (offs[i],) for i in range(nb.value)]

    def stats(self):
        nt = ctypes.c_int64()
        fl = ctypes.c_double()
        by = (ctypes.c_double * 3)()
        self.ctx.check(_lib.heff_task_stats(self._h, ctypes.byref(nt), ctypes.byref(fl), by))
        return dict(n_tasks=nt.value, flops=fl.value, bytes={"fp64": by[0], "fp32": by[1], "bf16x3": by[2]})

    def shard(self, rank, nranks):
        """Restrict every later product to the output blocks of `rank` of
        `nranks` (nranks = 1: the full product); returns the rank's
        algorithmic flops per product."""
        fl = ctypes.c_double()
        self.ctx.check(_lib.heff_blocks_shard(self.ctx._h, self._h, int(rank), int(nranks), ctypes.byref(fl)))
        return fl.value

    def variant_stats(self):
        """[(algorithmic flops per product, work-groups)] per kernel variant."""
        out = []
        for v in range(N_VARIANTS):
            fl = ctypes.c_double()
            nw = ctypes.c_int64()
            self.ctx.check(_lib.heff_task_stats_variant(self._h, v, ctypes.byref(fl), ctypes.byref(nw)))
            out.append((fl.value, nw.value))
        return out

    def issued_stats(self):
        """[(matrix-instruction flops, pipeline steps, steps of the longest
        work-group)] per kernel variant of the FP64/FP32 kernel."""
        out = []
        for v in range(N_VARIANTS):
            fl = ctypes.c_double()
            ns = ctypes.c_int64()
            mx = ctypes.c_int64()
            self.ctx.check(_lib.heff_task_stats_issued(self._h, v, ctypes.byref(fl), ctypes.byref(ns), ctypes.byref(mx)))
            out.append((fl.value, ns.value, mx.value))
        return out

    def energy(self, psi, prec=FP64):
        """<psi|H_eff|psi> (psi: device tensor of the precision's dtype)."""
        self._check_vec(psi, prec)
        e = ctypes.c_double()
        self.ctx.check(_lib.heff_energy(self.ctx._h, self._h, prec, _ptr(psi), ctypes.byref(e)))
        return e.value

    def energy_noalloc(self, psi, prec=FP64):
        """<psi|H_eff|psi> through heff_energy_noalloc: the same result as
        energy() without any device allocation (static scratch; psi of at
        most 6291456 FP64 / 12582912 FP32 elements)."""
        self._check_vec(psi, prec)
        e = ctypes.c_double()
        self.ctx.check(_lib.heff_energy_noalloc(self.ctx._h, self._h, prec, _ptr(psi), ctypes.byref(e)))
        return e.value

    def op_arena(self, prec=FP64):
        """torch views [left store, left temporaries, right store, right
        temporaries] of the operand arenas (library memory, no copy)."""
        import torch
        ptr = (_vp * 4)()
        n = (ctypes.c_int64 * 4)()
        self.ctx.check(_lib.heff_op_arena(self._h, prec, ptr, n))
        ts = "<f8" if prec == FP64 else "<f4"
        out = []
        for i in range(4):
            if n[i] == 0 or not ptr[i]:
                out.append(torch.empty(0, dtype=torch.float64 if prec == FP64 else torch.float32, device="cuda"))
            else:
                out.append(torch.as_tensor(_DeviceArray(ptr[i], n[i], ts, self), device="cuda"))
        return out

    def energy_backward(self, psi, gE=1.0, prec=FP64, ops=True):
        """(dE/dpsi, dE/d[left store | left temps], dE/d[right store | right
        temps]) scaled by gE; the operand gradients are None if ops is False."""
        import torch
        self._check_vec(psi, prec)
        dt = torch.float64 if prec == FP64 else torch.float32
        dpsi = torch.empty_like(psi)
        dL = dR = None
        if ops:
            n = (ctypes.c_int64 * 4)()
            ptr = (_vp * 4)()
            self.ctx.check(_lib.heff_op_arena(self._h, prec, ptr, n))
            dL = torch.empty(max(1, n[0] + n[1]), dtype=dt, device="cuda")
            dR = torch.empty(max(1, n[2] + n[3]), dtype=dt, device="cuda")
        self.ctx.check(_lib.heff_energy_backward(self.ctx._h, self._h, prec, _ptr(psi), float(gE), _ptr(dpsi),
                                                 _ptr(dL) if dL is not None else None,
                                                 _ptr(dR) if dR is not None else None))
        return dpsi, dL, dR

    def _check_vec(self, psi, prec):
        import torch
        want = torch.float64 if prec == FP64 else torch.float32
        if psi.dtype != want or psi.numel() != self.n_elem or not psi.is_cuda or not psi.is_contiguous():
            raise ValueError("psi must be a contiguous %s device tensor of %d elements" % (want, self.n_elem))

    def apply(self, psi, out, prec=FP64):
        """out = H_eff psi (device tensors: float64 for FP64, float32 otherwise)."""
        import torch
        want = torch.float64 if prec == FP64 else torch.float32
        if psi.dtype != want or out.dtype != want or psi.numel() != self.n_elem or out.numel() != self.n_elem:
            raise ValueError("psi/out must be %s tensors of %d elements" % (want, self.n_elem))
        if not (psi.is_cuda and out.is_cuda and psi.is_contiguous() and out.is_contiguous()):
            raise ValueError("psi/out must be contiguous device tensors")
        self.ctx.check(_lib.heff_apply(self.ctx._h, self._h, prec, _ptr(psi), _ptr(out)))
        return out

    def diag(self, out):
        self.ctx.check(_lib.heff_diag(self.ctx._h, self._h, _ptr(out)))
        return out

    def truncate(self, psi, d_keep):
        """Keep the d_keep largest singular values of psi over the enlarged
        left sectors.  Returns dict(sing, discarded, tab {(nu, nd): dim},
        iso: {(nu, nd): stacked matrix}) (isometry copied to the host)."""
        import torch
        if psi.dtype != torch.float64 or psi.numel() != self.n_elem or not psi.is_cuda:
            raise ValueError("psi must be a float64 device tensor of %d elements" % self.n_elem)
        h = _vp()
        self.ctx.check(_lib.heff_truncate(self.ctx._h, self._h, _ptr(psi), int(d_keep), ctypes.byref(h)))
        try:
            return _trunc_dict(self.ctx, h, psi.device)
        finally:
            _lib.heff_trunc_free(h)

    def sweep_right(self, psi, d_keep, precs=None):
        """One left-to-right sweep step from these blocks (built with
        keep_env=True) and the optimized two-site vector psi (float64 device
        tensor): truncation to d_keep states, Ren_l, the pair one site to the
        right.  Returns (blocks of the new pair, its start vector as a float64
        device tensor viewing memory owned by those blocks, truncation dict
        as truncate())."""
        import torch
        if psi.dtype != torch.float64 or psi.numel() != self.n_elem or not psi.is_cuda:
            raise ValueError("psi must be a float64 device tensor of %d elements" % self.n_elem)
        precs = self.precs if precs is None else tuple(precs)
        mask = 0
        for pr in precs:
            mask |= 1 << pr
        out = _vp()
        tr = _vp()
        self.ctx.check(_lib.heff_sweep_right(self.ctx._h, self._h, _ptr(psi), int(d_keep), mask, ctypes.byref(out),
                                             ctypes.byref(tr)))
        try:
            info = _trunc_dict(self.ctx, tr, psi.device)
        finally:
            _lib.heff_trunc_free(tr)
        nb = Blocks(self.ctx, None, precs=precs, _handle=out)
        sp = ctypes.POINTER(ctypes.c_double)()
        self.ctx.check(_lib.heff_start_vector(out, ctypes.byref(sp)))
        addr = ctypes.cast(sp, ctypes.c_void_p).value
        start = torch.as_tensor(_DeviceArray(addr, nb.n_elem, "<f8", nb), device=psi.device)
        return nb, start, info

    def _check64(self, psi):
        import torch
        if psi.dtype != torch.float64 or psi.numel() != self.n_elem or not psi.is_cuda or not psi.is_contiguous():
            raise ValueError("psi must be a contiguous float64 device tensor of %d elements" % self.n_elem)

    def rotate_pair(self, psi, theta, out=None):
        """The vector of the same state after the rotation of the pair's two
        orbitals by theta (heff_rotate_pair)."""
        import torch
        self._check64(psi)
        out = torch.empty_like(psi) if out is None else out
        self.ctx.check(_lib.heff_rotate_pair(self.ctx._h, self._h, float(theta), _ptr(psi), _ptr(out)))
        return out

    def pair_entropy(self, psi):
        """(S_1/2, S_1) of the left part of the normalized state psi."""
        self._check64(psi)
        sh, sv = ctypes.c_double(), ctypes.c_double()
        self.ctx.check(_lib.heff_pair_entropy(self.ctx._h, self._h, _ptr(psi), ctypes.byref(sh), ctypes.byref(sv)))
        return sh.value, sv.value

    def optimize_pair(self, psi):
        """Mode rotation of the pair minimizing S_1/2: (theta, rotated psi,
        S_1/2 before, S_1/2 after, trials)."""
        import torch
        self._check64(psi)
        out = torch.empty_like(psi)
        th, sb, sa = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        ne = ctypes.c_int32()
        self.ctx.check(_lib.heff_optimize_pair(self.ctx._h, self._h, _ptr(psi), _ptr(out), ctypes.byref(th),
                                               ctypes.byref(sb), ctypes.byref(sa), ctypes.byref(ne)))
        return th.value, out, sb.value, sa.value, ne.value

    def debug_op(self, side, kind, i=0, j=0):
        n = _lib.heff_debug_op(self._h, side, kind, i, j, None, 0)
        if n <= 0:
            return None
        buf = np.empty(n, dtype=np.float64)
        got = _lib.heff_debug_op(self._h, side, kind, i, j, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n)
        if got != n:
            raise HeffError(-4, "debug copy failed")
        return buf

    def close(self):
        if getattr(self, "_h", None):
            _lib.heff_blocks_free(self._h)
            self._h = None

    def __del__(self, _fin=sys.is_finalizing):
        if _fin():  # the HIP runtime may already be gone
            return
        try:
            self.close()
        except Exception:
            pass


class Davidson:
    """Device Davidson for the lowest eigenpair of H_eff."""

    def __init__(self, blocks: Blocks, psi0, m_max=24, tol=1e-10):
        self.blocks = blocks
        self.tol = tol
        self.ctx = blocks.ctx
        h = _vp()
        self.ctx.check(_lib.heff_dav_create(self.ctx._h, blocks._h, m_max, tol, _ptr(psi0), ctypes.byref(h)))
        self._h = h
        self.converged = False

    def step(self, prec=FP64):
        th = ctypes.c_double()
        rn = ctypes.c_double()
        self.ctx.check(_lib.heff_davidson_step(self.ctx._h, self._h, prec, ctypes.byref(th), ctypes.byref(rn)))
        self.theta, self.resid = th.value, rn.value
        self.converged = rn.value <= self.tol * abs(th.value)
        return th.value, rn.value

    def ritz(self, out):
        self.ctx.check(_lib.heff_dav_ritz(self.ctx._h, self._h, _ptr(out)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.heff_dav_free(self._h)
            self._h = None

    def __del__(self, _fin=sys.is_finalizing):
        if _fin():  # the HIP runtime may already be gone
            return
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent problems (FP32 operands) in one persistent, graph-captured
    launch per kernel variant.  x / y are the concatenated FP32 input and
    output device vectors; views(i) gives problem i's slices."""

    def __init__(self, ctx: Context, blocks):
        import torch
        self.ctx = ctx
        self.blocks = list(blocks)
        arr = (_vp * len(self.blocks))(*[b._h for b in self.blocks])
        self._arr = arr
        n = len(self.blocks)
        offs = (ctypes.c_int64 * n)()
        tot = ctypes.c_int64()
        ctx.check(_lib.heff_batch_layout(arr, n, offs, ctypes.byref(tot)))
        self.offsets = list(offs)
        self.n_total = tot.value
        self.x = torch.zeros(max(self.n_total, 1), dtype=torch.float32, device="cuda")
        self.y = torch.zeros(max(self.n_total, 1), dtype=torch.float32, device="cuda")
        h = _vp()
        ctx.check(_lib.heff_batch_create(ctx._h, arr, n, _ptr(self.x), _ptr(self.y), ctypes.byref(h)))
        self._h = h
        if self.io() != (self.offsets, self.n_total):
            raise HeffError(-1, "batch layout and batch object disagree")

    def io(self):
        """(offsets, n_total) of the concatenated input/output vectors as the
        batch object holds them."""
        po = ctypes.POINTER(ctypes.c_int64)()
        tot = ctypes.c_int64()
        self.ctx.check(_lib.heff_batch_io(self._h, ctypes.byref(po), ctypes.byref(tot)))
        return [po[i] for i in range(len(self.blocks))], tot.value

    def views(self, i):
        o, n = self.offsets[i], self.blocks[i].n_elem
        return self.x[o:o + n], self.y[o:o + n]

    def set_grid(self, grid):
        g = (ctypes.c_int32 * N_VARIANTS)(*grid)
        self.ctx.check(_lib.heff_batch_set_grid(self._h, g))

    def stats(self):
        fl = ctypes.c_double()
        g = (ctypes.c_int32 * N_VARIANTS)()
        w = (ctypes.c_int64 * N_VARIANTS)()
        self.ctx.check(_lib.heff_batch_stats(self._h, ctypes.byref(fl), g, w))
        return dict(flops=fl.value, grid=list(g), work_items=list(w))

    def apply(self, use_graph=True):
        self.ctx.check(_lib.heff_batch_apply(self.ctx._h, self._h, 1 if use_graph else 0))

    def close(self):
        if getattr(self, "_h", None):
            _lib.heff_batch_free(self._h)
            self._h = None

    def __del__(self, _fin=sys.is_finalizing):
        if _fin():
            return
        try:
            self.close()
        except Exception:
            pass


def rotate_integrals(h, V, x, y, theta):
    """(U^T h U, V rotated on all four indices) for the rotation of orbitals
    (x, y) by theta (heff_rotate_integrals; host only)."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    n = h.shape[0]
    h2 = np.empty_like(h)
    V2 = np.empty_like(V)
    rc = _lib.heff_rotate_integrals(n, h.ctypes.data, V.ctypes.data, int(x), int(y), float(theta),
                                    h2.ctypes.data, V2.ctypes.data)
    if rc != 0:
        raise HeffError(rc, "heff_rotate_integrals failed")
    return h2, V2


def kappa_gradient(ctx: Context, problem, psi, pairs):
    """Orbital-rotation gradient g_xy = dE/dkappa_xy of E = <psi|H_eff|psi>
    (psi: float64 device tensor; isometries and psi fixed) for the given
    orbital pairs; one block build and one product per pair (E is linear in
    the integrals)."""
    keep = []
    prob = _marshal(problem, keep)
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1))
    g = np.zeros(len(pr) // 2)
    ctx.check(_lib.heff_kappa_gradient(ctx._h, ctypes.byref(prob), _ptr(psi), len(pr) // 2,
                                       pr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return g


def integral_gradient(ctx: Context, problem, psi, one_body=True, two_body=True):
    """(dE/dh, dE/dV) of E = <psi|H_eff|psi> (psi: float64 device tensor;
    isometries and psi fixed) as symmetric tensors: the spin-summed
    one-particle density matrix and half the symmetrized two-particle one of
    the two-site state.  Exact; one block build and one product per
    symmetry orbit of integral indices (small orbital counts)."""
    keep = []
    prob = _marshal(problem, keep)
    n = problem.n_orb
    gh = np.zeros((n, n)) if one_body else None
    gV = np.zeros((n,) * 4) if two_body else None
    dp = ctypes.POINTER(ctypes.c_double)
    ctx.check(_lib.heff_integral_gradient(ctx._h, ctypes.byref(prob), _ptr(psi),
                                          gh.ctypes.data_as(dp) if gh is not None else None,
                                          gV.ctypes.data_as(dp) if gV is not None else None))
    return gh, gV


def _energy_function():
    import torch

    class HeffEnergy(torch.autograd.Function):
        """E = <psi|H_eff|psi> as a differentiable function of psi and of the
        four operand arenas (views from Blocks.op_arena, whose memory the
        product reads).  Usage: HeffEnergy.apply(psi, L0, L1, R0, R1, blocks,
        prec)."""

        @staticmethod
        def forward(ctx_, psi, L0, L1, R0, R1, blocks, prec):
            ctx_.blocks, ctx_.prec = blocks, prec
            ctx_.sizes = (L0.numel(), L1.numel(), R0.numel(), R1.numel())
            ctx_.save_for_backward(psi)
            return torch.tensor(blocks.energy(psi.detach(), prec), dtype=torch.float64, device=psi.device)

        @staticmethod
        def backward(ctx_, gE):
            (psi,) = ctx_.saved_tensors
            need_ops = any(ctx_.needs_input_grad[1:5])
            dpsi, dL, dR = ctx_.blocks.energy_backward(psi.detach(), float(gE), ctx_.prec, ops=need_ops)
            n0, n1, n2, n3 = ctx_.sizes
            gl = [None] * 4
            if need_ops:
                gl = [dL[:n0], dL[n0:n0 + n1], dR[:n2], dR[n2:n2 + n3]]
            return (dpsi, gl[0], gl[1], gl[2], gl[3], None, None)

    return HeffEnergy


def _integral_energy_function():
    import dataclasses

    import torch

    class HeffIntegralEnergy(torch.autograd.Function):
        """E = <psi|H_eff(h, V)|psi> as a differentiable function of psi and
        of the integrals h (n x n) and V (n^4, (ij|kl)); the isometries of
        `problem` are held fixed.  The forward builds the blocks from h and
        V; the backward gives dE/dpsi = 2 H_eff psi and, when asked for,
        dE/dh and dE/dV by heff_integral_gradient (the one- and half the
        two-particle density matrix of the state: exact, one build per
        symmetry orbit of integral indices, meant for small orbital counts).
        Usage: HeffIntegralEnergy.apply(psi, h, V, problem, context)."""

        @staticmethod
        def forward(ctx_, psi, h, V, problem, context):
            hp = h.detach().double().cpu().numpy()
            Vp = V.detach().double().cpu().numpy()
            prob = dataclasses.replace(problem, h=hp, V=Vp)
            B = Blocks(context, prob)
            ctx_.blocks, ctx_.problem, ctx_.context = B, prob, context
            ctx_.save_for_backward(psi, h, V)
            return torch.tensor(B.energy(psi.detach()), dtype=torch.float64, device=psi.device)

        @staticmethod
        def backward(ctx_, gE):
            psi, h, V = ctx_.saved_tensors
            g = float(gE)
            dpsi = dh = dV = None
            if ctx_.needs_input_grad[0]:
                dpsi, _, _ = ctx_.blocks.energy_backward(psi.detach(), g, FP64, ops=False)
            nh, nv = ctx_.needs_input_grad[1], ctx_.needs_input_grad[2]
            if nh or nv:
                gh, gV = integral_gradient(ctx_.context, ctx_.problem, psi.detach(), one_body=nh, two_body=nv)
                if nh:
                    dh = torch.as_tensor(g * gh, dtype=h.dtype, device=h.device)
                if nv:
                    dV = torch.as_tensor(g * gV, dtype=V.dtype, device=V.device)
            return dpsi, dh, dV, None, None

    return HeffIntegralEnergy


_HIE = None


def heff_integral_energy_function():
    """The torch.autograd.Function of E(psi, h, V) (created lazily)."""
    global _HIE
    if _HIE is None:
        _HIE = _integral_energy_function()
    return _HIE


_HE = None


def heff_energy_function():
    """The torch.autograd.Function of E = <psi|H_eff|psi> (created lazily so
    that importing this module does not import torch)."""
    global _HE
    if _HE is None:
        _HE = _energy_function()
    return _HE


# --------------------------------------------------------------------------
# SU(2) spin-adapted product
# --------------------------------------------------------------------------
def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_I32P)


def _su2_block(blk, keep):
    """heff_su2_block from a synth_su2 Block (arrays kept alive in keep)."""
    from . import synth_su2
    sec = np.array(blk.sectors, dtype=np.int32).reshape(-1, 3)
    cols = [np.ascontiguousarray(sec[:, j]) for j in range(3)]
    two_k = np.array([op[0] for op in blk.ops], dtype=np.int32)
    dn = np.array([op[1] for op in blk.ops], dtype=np.int32)
    bop, bout, bin_, boff, data = synth_su2.op_arrays(blk)
    data = np.ascontiguousarray(data, dtype=np.float64)
    boff = np.ascontiguousarray(boff, dtype=np.int64)
    keep += cols + [two_k, dn, bop, bout, bin_, boff, data]
    b = _Su2Block()
    b.n_sect = len(blk.sectors)
    b.n, b.two_s, b.dim = (c.ctypes.data_as(_I32P) for c in cols)
    b.n_ops = len(blk.ops)
    b.two_k, b.dn = two_k.ctypes.data_as(_I32P), dn.ctypes.data_as(_I32P)
    b.n_blk = len(bop)
    b.blk_op, b.blk_out, b.blk_in = (x.ctypes.data_as(_I32P) for x in (bop, bout, bin_))
    b.blk_off = boff.ctypes.data_as(_I64P)
    b.data = data.ctypes.data_as(_F64P)
    b.data_len = data.size
    return b


def _su2_marshal(problem, keep):
    pr = _Su2Problem()
    pr.left = _su2_block(problem.L, keep)
    pr.right = _su2_block(problem.R, keep)
    t = problem.terms
    cols = [np.array([x[j] for x in t], dtype=np.int32) for j in range(5)]
    coef = np.array([x[5] for x in t], dtype=np.float64)
    keep += cols + [coef]
    pr.n_terms = len(t)
    pr.term_l, pr.term_site_k, pr.term_site_k1, pr.term_r, pr.term_two_s = (c.ctypes.data_as(_I32P) for c in cols)
    pr.term_coef = coef.ctypes.data_as(_F64P)
    pr.n_tot, pr.two_s_tot = problem.n_tot, problem.ts_tot
    return pr


def su2_factor(two_j):
    """F(a, b, c; k_a, k_b, k_c; a', b', c') of doubled spins (host only)."""
    arr, ptr = _i32(list(two_j))
    if arr.size != 9:
        raise ValueError("nine doubled spins")
    f = ctypes.c_double()
    rc = _lib.heff_su2_factor(ptr, ctypes.byref(f))
    if rc != 0:
        raise HeffError(rc, "heff_su2_factor")
    return f.value


class Su2:
    """SU(2) spin-adapted two-site product of a synth_su2 problem."""

    def __init__(self, ctx: Context, problem, precs=(FP64,)):
        self.ctx = ctx
        keep = []
        pr = _su2_marshal(problem, keep)
        mask = 0
        for p in precs:
            mask |= 1 << p
        out = _vp()
        ctx.check(_lib.heff_su2_create(ctx._h, ctypes.byref(pr), mask, ctypes.byref(out)))
        self._h = out
        n = ctypes.c_int64()
        nb = ctypes.c_int32()
        desc = _I32P()
        offs = _I64P()
        ctx.check(_lib.heff_su2_layout(out, ctypes.byref(n), ctypes.byref(nb), ctypes.byref(desc), ctypes.byref(offs)))
        self.n_elem = n.value
        self.blocks = [(tuple(desc[8 * i + j] for j in range(6)), offs[i], desc[8 * i + 6], desc[8 * i + 7])
                       for i in range(nb.value)]

    def stats(self):
        nt = ctypes.c_int64()
        fl = ctypes.c_double()
        nr = ctypes.c_double()
        self.ctx.check(_lib.heff_su2_stats(self._h, ctypes.byref(nt), ctypes.byref(fl), ctypes.byref(nr)))
        return dict(n_tasks=nt.value, flops=fl.value, n_resolved=nr.value)

    def apply(self, psi, out, prec=FP64):
        import torch
        want = torch.float64 if prec == FP64 else torch.float32
        if psi.dtype != want or out.dtype != want or psi.numel() != self.n_elem or out.numel() != self.n_elem:
            raise ValueError("psi/out must be %s tensors of %d elements" % (want, self.n_elem))
        if not (psi.is_cuda and out.is_cuda and psi.is_contiguous() and out.is_contiguous()):
            raise ValueError("psi/out must be contiguous device tensors")
        self.ctx.check(_lib.heff_su2_apply(self.ctx._h, self._h, prec, _ptr(psi), _ptr(out)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.heff_su2_free(self._h)
            self._h = None

    def __del__(self, _fin=sys.is_finalizing):
        if _fin():
            return
        try:
            self.close()
        except Exception:
            pass
