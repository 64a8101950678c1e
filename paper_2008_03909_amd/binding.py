"""Thin Python binding of ``libconnectit_hip.so`` (C ABI: include/connectit_hip.h).

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step runs in the library's kernels.  If the
library is missing this module raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "libconnectit_hip.so")

CC_OK, CC_EINVAL, CC_ENOMEM, CC_EDEVICE, CC_ELIVELOCK, CC_EBUSY, CC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
SAMPLE_NONE, SAMPLE_KOUT, SAMPLE_BFS, SAMPLE_LDD = 0, 1, 2, 3
KOUT_HYBRID, KOUT_AFFOREST, KOUT_PURE, KOUT_MAXDEG = 0, 1, 2, 3
FIN_UF_REM_CAS, FIN_UF_ASYNC, FIN_SV, FIN_LT = 0, 1, 2, 3
FIN_UF_EARLY, FIN_UF_HOOKS, FIN_LP = 4, 5, 6
FIND_NAIVE, FIND_ATOMIC_SPLIT, FIND_ATOMIC_HALVE, FIND_COMPRESS = 0, 1, 2, 3
SPLICE_SPLIT_ONE, SPLICE_HALVE_ONE, SPLICE_ATOMIC = 0, 1, 2
LT_CONNECT, LT_PARENT_CONNECT, LT_EXTENDED_CONNECT, LT_ROOTUP, LT_FULL_SHORTCUT, LT_ALTER = 0, 1, 2, 4, 8, 16
LT_CRSA = LT_CONNECT | LT_ROOTUP | LT_ALTER
LT_PRSA = LT_PARENT_CONNECT | LT_ROOTUP | LT_ALTER
LT_PRS = LT_PARENT_CONNECT | LT_ROOTUP
LT_CRFA = LT_CONNECT | LT_ROOTUP | LT_FULL_SHORTCUT | LT_ALTER
LT_PRFA = LT_PARENT_CONNECT | LT_ROOTUP | LT_FULL_SHORTCUT | LT_ALTER
LT_PRF = LT_PARENT_CONNECT | LT_ROOTUP | LT_FULL_SHORTCUT
LT_NAMES = {LT_CRSA: "CRSA", LT_PRSA: "PRSA", LT_PRS: "PRS", LT_CRFA: "CRFA", LT_PRFA: "PRFA", LT_PRF: "PRF"}
# the non-root-based variants (appendix "Liu-Tarjan Algorithms")
LT_NONROOT = {
    "CUSA": LT_CONNECT | LT_ALTER, "PUSA": LT_PARENT_CONNECT | LT_ALTER, "PUS": LT_PARENT_CONNECT,
    "EUSA": LT_EXTENDED_CONNECT | LT_ALTER, "EUS": LT_EXTENDED_CONNECT,
    "CUFA": LT_CONNECT | LT_FULL_SHORTCUT | LT_ALTER, "PUFA": LT_PARENT_CONNECT | LT_FULL_SHORTCUT | LT_ALTER,
    "PUF": LT_PARENT_CONNECT | LT_FULL_SHORTCUT, "EUFA": LT_EXTENDED_CONNECT | LT_FULL_SHORTCUT | LT_ALTER,
    "EUF": LT_EXTENDED_CONNECT | LT_FULL_SHORTCUT,
}
LT_NAMES.update({r: name for name, r in LT_NONROOT.items()})


class cc_variant(ctypes.Structure):
    _fields_ = [
        ("sample", ctypes.c_int32),
        ("kout_k", ctypes.c_int32),
        ("kout_mode", ctypes.c_int32),
        ("bfs_tries", ctypes.c_int32),
        ("ldd_beta", ctypes.c_float),
        ("ldd_permute", ctypes.c_int32),
        ("finish", ctypes.c_int32),
        ("find", ctypes.c_int32),
        ("splice", ctypes.c_int32),
        ("lt_rules", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
    ]

    def copy(self, **kw) -> "cc_variant":
        v = cc_variant()
        ctypes.memmove(ctypes.byref(v), ctypes.byref(self), ctypes.sizeof(cc_variant))
        for k, x in kw.items():
            setattr(v, k, x)
        return v

    def name(self) -> str:
        s = {0: "none", 1: "kout", 2: "bfs", 3: "ldd"}[self.sample]
        if self.sample == SAMPLE_KOUT:
            s += {0: "", 1: "-afforest", 2: "-pure", 3: "-maxdeg"}[self.kout_mode] + f"(k={self.kout_k})"
        if self.finish == FIN_UF_REM_CAS:
            f = "rem-cas/" + ["split-one", "halve-one", "splice"][self.splice] + "/" + \
                ["naive", "split", "halve"][self.find]
        elif self.finish in (FIN_UF_ASYNC, FIN_UF_EARLY, FIN_UF_HOOKS):
            f = {FIN_UF_ASYNC: "async/", FIN_UF_EARLY: "early/", FIN_UF_HOOKS: "hooks/"}[self.finish] + \
                ["naive", "split", "halve", "compress"][self.find]
        elif self.finish == FIN_LP:
            f = "lp"
        elif self.finish == FIN_SV:
            f = "sv"
        else:
            f = "lt-" + LT_NAMES.get(self.lt_rules, str(self.lt_rules))
        return f"{s}+{f}"

    def __repr__(self):
        return f"cc_variant({self.name()}, seed={self.seed})"


class cc_amsf_options(ctypes.Structure):
    _fields_ = [("epsilon", ctypes.c_float), ("light_fraction", ctypes.c_float), ("seed", ctypes.c_uint64)]


class cc_stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("m", ctypes.c_int64),
        ("lmax", ctypes.c_int32), ("sample_success", ctypes.c_int32),
        ("lmax_size", ctypes.c_int64), ("candidates", ctypes.c_int64),
        ("candidate_edges", ctypes.c_int64),
        ("sample_rounds", ctypes.c_int32), ("finish_rounds", ctypes.c_int32),
        ("num_components", ctypes.c_int64),
        ("sample_bottom_up", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class cc_csr_report(ctypes.Structure):
    _fields_ = [
        ("failed", ctypes.c_uint32), ("rows_sorted", ctypes.c_int32),
        ("symmetry_checked", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("bad_entries", ctypes.c_int64), ("first_bad_row", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


CSR_OFFSET0, CSR_OFFSETN, CSR_MONOTONE, CSR_ID_RANGE, CSR_ASYMMETRIC = 1, 2, 4, 8, 16

_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int


def lib():
    """The loaded library.  Raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(f"{SO_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(SO_PATH)
        sig = {
            "cc_ctx_create": (_int, [_int, ctypes.POINTER(_vp)]),
            "cc_ctx_destroy": (None, [_vp]),
            "cc_ctx_sync_status": (_int, [_vp]),
            "cc_last_stats": (_int, [_vp, ctypes.POINTER(cc_stats)]),
            "cc_ctx_set_timing": (_int, [_vp, _int]),
            "cc_ctx_set_round_limit": (_int, [_vp, ctypes.c_int32]),
            "cc_ctx_set_timing_phase": (_int, [_vp, ctypes.c_char_p]),
            "cc_phase_times": (_int, [_vp, _int, ctypes.POINTER(ctypes.c_char_p),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]),
            "cc_phase_times_reset": (None, [_vp]),
            "cc_default_variant": (_int, [ctypes.POINTER(cc_variant)]),
            "cc_check_variant": (_int, [ctypes.POINTER(cc_variant)]),
            "cc_workspace_bytes": (_int, [_i64, _i64, ctypes.POINTER(cc_variant), ctypes.POINTER(ctypes.c_size_t)]),
            "cc_connectivity_csr": (_int, [_vp, _i64, _i64, _vp, _int, _vp, ctypes.POINTER(cc_variant), _vp,
                                           ctypes.c_size_t, _vp, _vp, _vp]),
            "cc_mapped_workspace_bytes": (_int, [_i64, _i64, ctypes.POINTER(cc_variant),
                                                 ctypes.POINTER(ctypes.c_size_t)]),
            "cc_connectivity_csr_mapped": (_int, [_vp, _i64, _i64, _i64, _vp, _int, _vp, _vp, _vp,
                                                  ctypes.POINTER(cc_variant), _vp, ctypes.c_size_t, _vp, _vp, _vp]),
            "cc_csr_active_prefix": (_int, [_i64, _vp, _int, _vp, _vp]),
            "cc_noalloc_scratch_bytes": (ctypes.c_size_t, []),
            "cc_connectivity_csr_noalloc": (_int, [_vp, _i64, _i64, _vp, _int, _vp, ctypes.POINTER(cc_variant), _vp,
                                                   _vp, _vp]),
            "cc_sample_csr": (_int, [_vp, _i64, _i64, _vp, _int, _vp, ctypes.POINTER(cc_variant), _vp,
                                     ctypes.c_size_t, _vp, ctypes.POINTER(ctypes.c_int32), _vp]),
            "cc_coo_workspace_bytes": (_int, [_i64, _i64, ctypes.POINTER(cc_variant),
                                              ctypes.POINTER(ctypes.c_size_t)]),
            "cc_connectivity_coo": (_int, [_vp, _i64, _i64, _vp, _vp, ctypes.POINTER(cc_variant), _vp,
                                           ctypes.c_size_t, _vp, _vp, _vp]),
            "cc_forest_workspace_bytes": (_int, [_i64, _i64, ctypes.POINTER(cc_variant),
                                                 ctypes.POINTER(ctypes.c_size_t)]),
            "cc_spanning_forest_csr": (_int, [_vp, _i64, _i64, _vp, _int, _vp, ctypes.POINTER(cc_variant), _vp,
                                              ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp]),
            "cc_forest_mapped_workspace_bytes": (_int, [_i64, _i64, ctypes.POINTER(cc_variant),
                                                        ctypes.POINTER(ctypes.c_size_t)]),
            "cc_spanning_forest_csr_mapped": (_int, [_vp, _i64, _i64, _i64, _vp, _int, _vp, _vp, _vp,
                                                     ctypes.POINTER(cc_variant), _vp, ctypes.c_size_t, _vp, _vp, _vp,
                                                     _vp, _vp]),
            "cc_amsf_default_options": (_int, [ctypes.POINTER(cc_amsf_options)]),
            "cc_amsf_workspace_bytes": (_int, [_i64, _i64, ctypes.POINTER(cc_amsf_options),
                                               ctypes.POINTER(ctypes.c_size_t)]),
            "cc_amsf_csr": (_int, [_vp, _i64, _i64, _vp, _int, _vp, _vp, ctypes.POINTER(cc_amsf_options), _vp,
                                   ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "cc_amsf_mapped_workspace_bytes": (_int, [_i64, _i64, ctypes.POINTER(cc_amsf_options),
                                                      ctypes.POINTER(ctypes.c_size_t)]),
            "cc_amsf_csr_mapped": (_int, [_vp, _i64, _i64, _i64, _vp, _int, _vp, _vp, _vp, _vp,
                                          ctypes.POINTER(cc_amsf_options), _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp,
                                          _vp, _vp, _vp]),
            "cc_validate_csr": (_int, [_vp, _i64, _i64, _vp, _int, _vp, _int, ctypes.POINTER(cc_csr_report), _vp]),
            "cc_csr_workspace_bytes": (_int, [_i64, _i64, ctypes.POINTER(ctypes.c_size_t)]),
            "cc_build_csr": (_int, [_vp, _i64, _i64, _vp, _vp, _int, _vp, ctypes.c_size_t, _vp, _int, _vp, _vp,
                                    _vp]),
            "cc_csr_degree_order_workspace_bytes": (_int, [_i64, _i64, ctypes.POINTER(ctypes.c_size_t)]),
            "cc_build_csr_degree_order": (_int, [_vp, _i64, _i64, _vp, _vp, _int, _vp, ctypes.c_size_t, _vp, _int,
                                                 _vp, _vp, _vp, _vp, _vp]),
            "cc_stream_create": (_int, [_vp, _i64, ctypes.POINTER(cc_variant), ctypes.POINTER(_vp)]),
            "cc_stream_destroy": (None, [_vp]),
            "cc_stream_init_csr": (_int, [_vp, _i64, _vp, _int, _vp, _vp, ctypes.c_size_t, _vp]),
            "cc_insert_batch": (_int, [_vp, _i64, _vp, _vp, _vp]),
            "cc_query_batch": (_int, [_vp, _i64, _vp, _vp, _vp, _vp]),
            "cc_stream_labels": (_int, [_vp, _vp, _vp, _vp]),
            "cc_process_batch": (_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp]),
            "cc_stream_type": (ctypes.c_int32, [_vp]),
            "cc_stream_sync_status": (_int, [_vp]),
            "cc_server_create": (_int, [_vp, _i64, ctypes.POINTER(cc_variant), _i64, _int, _int, ctypes.POINTER(_vp)]),
            "cc_server_destroy": (None, [_vp]),
            "cc_server_clock": (ctypes.c_double, [_vp]),
            "cc_server_submit_insert": (_int, [_vp, _i64, _vp, _vp, ctypes.c_double, ctypes.POINTER(_i64)]),
            "cc_server_submit_query": (_int, [_vp, _i64, _vp, _vp, _vp, ctypes.c_double, ctypes.POINTER(_i64)]),
            "cc_server_poll": (_int, [_vp, _int]),
            "cc_server_run_trace": (_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "cc_server_request_info": (_int, [_vp, _i64, ctypes.POINTER(_int), ctypes.POINTER(ctypes.c_double)]),
            "cc_server_labels": (_int, [_vp, _vp, _vp, _vp]),
            "cc_server_pool_used": (_i64, [_vp]),
            "cc_server_stamped": (ctypes.c_int32, [_vp]),
            "cc_server_event_count": (_i64, [_vp]),
            "cc_mlp_param_count": (_i64, [ctypes.c_int32]),
            "cc_mlp_forward": (_int, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp]),
            "cc_mlp_backward": (_int, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "cc_mlp_adam": (_int, [_vp, _vp, _vp, _vp, _vp, _i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_int32, _vp]),
            "cc_mlp_pack_bf16": (_int, [_vp, _vp, _i64, _vp]),
            "cc_graph_features": (_int, [_vp, _i64, _i64, _vp, _int, _vp, _vp, ctypes.c_size_t,
                                         ctypes.POINTER(ctypes.c_float), _vp]),
            "cc_connectivity_auto": (_int, [_vp, _i64, _i64, _vp, _int, _vp, _vp, ctypes.c_int32,
                                            ctypes.POINTER(cc_variant), ctypes.POINTER(ctypes.c_float), _vp,
                                            ctypes.c_size_t, _vp, _vp, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_float), _vp]),
            "cc_select_variant": (_int, [_vp, _i64, _i64, _vp, _int, _vp, _vp, ctypes.c_int32,
                                         ctypes.POINTER(cc_variant), ctypes.POINTER(ctypes.c_float), _vp,
                                         ctypes.c_size_t, ctypes.POINTER(cc_variant),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float), _vp]),
            "cc_ctx_set_selector_gate": (_int, [_vp, _i64, ctypes.c_int32]),
            "cc_calib_copy": (_int, [_vp, _vp, ctypes.c_size_t, _vp]),
            "cc_calib_workspace_bytes": (_int, [_i64, ctypes.POINTER(ctypes.c_size_t)]),
            "cc_calib_edges": (_int, [_i64, _i64, _vp, _int, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
            "cc_status_string": (ctypes.c_char_p, [_int]),
            "cc_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class CCError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.cc_last_error().decode(errors="replace")
        super().__init__(f"{where}: {L.cc_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def _check(status: int, where: str):
    if status != CC_OK:
        raise CCError(status, where)


def _ptr(t: torch.Tensor | None):
    """Device address of a tensor (NULL for None).  Host tensors are refused:
    the library dereferences these addresses in kernels."""
    if t is None:
        return ctypes.c_void_p(0)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_tensor(x, dtype, device):
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=dtype)
    else:
        t = torch.as_tensor(x, dtype=dtype, device=device)
    return t.contiguous()


def default_variant(**kw) -> cc_variant:
    v = cc_variant()
    _check(lib().cc_default_variant(ctypes.byref(v)), "cc_default_variant")
    for k, x in kw.items():
        setattr(v, k, x)
    return v


def check_variant(v: cc_variant) -> int:
    return lib().cc_check_variant(ctypes.byref(v))


def workspace_bytes(n: int, m: int, v: cc_variant) -> int:
    b = ctypes.c_size_t()
    _check(lib().cc_workspace_bytes(n, m, ctypes.byref(v), ctypes.byref(b)), "cc_workspace_bytes")
    return int(b.value)


class Context:
    """Owns a cc_ctx (device scalars, timing events)."""

    def __init__(self, device: int = 0):
        self.device = device
        self.h = ctypes.c_void_p()
        _check(lib().cc_ctx_create(device, ctypes.byref(self.h)), "cc_ctx_create")
        self._ws = None

    def close(self):
        if self.h:
            lib().cc_ctx_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def torch_device(self):
        return torch.device("cuda", self.device)

    def workspace(self, nbytes: int) -> torch.Tensor:
        """A cached device byte buffer of at least nbytes."""
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.torch_device)
        return self._ws

    def sync_status(self):
        _check(lib().cc_ctx_sync_status(self.h), "cc_ctx_sync_status")

    def last_stats(self) -> dict:
        s = cc_stats()
        _check(lib().cc_last_stats(self.h, ctypes.byref(s)), "cc_last_stats")
        return s.as_dict()

    def set_timing(self, on: bool, only: str | None = None):
        """Phase events on (every phase, or only the phase named `only`)."""
        _check(lib().cc_ctx_set_timing_phase(self.h, (only or "").encode()), "cc_ctx_set_timing_phase")
        _check(lib().cc_ctx_set_timing(self.h, int(on)), "cc_ctx_set_timing")

    def set_round_limit(self, limit: int):
        _check(lib().cc_ctx_set_round_limit(self.h, int(limit)), "cc_ctx_set_round_limit")

    def phase_times(self) -> dict:
        k = lib().cc_phase_times(self.h, 0, None, None, None)
        names = (ctypes.c_char_p * max(k, 1))()
        ms = (ctypes.c_double * max(k, 1))()
        cnt = (ctypes.c_int64 * max(k, 1))()
        k = lib().cc_phase_times(self.h, k, names, ms, cnt)
        return {names[i].decode(): (ms[i], cnt[i]) for i in range(k)}

    def phase_times_reset(self):
        lib().cc_phase_times_reset(self.h)


class CSR:
    """A device CSR: offsets (n+1, int32 or int64) and adj (m, int32)."""

    def __init__(self, n: int, offsets: torch.Tensor, adj: torch.Tensor):
        self.n = int(n)
        self.offsets = offsets
        self.adj = adj
        self.m = int(adj.numel())

    @property
    def o64(self) -> int:
        return int(self.offsets.dtype == torch.int64)


def build_csr(ctx: Context, n: int, u, v, dedup: bool = True, offsets_64bit: bool | None = None,
              stream=None) -> CSR:
    """cc_build_csr: symmetric, row-sorted CSR of an undirected pair list."""
    dev = ctx.torch_device
    ut = _dev_tensor(u, torch.int32, dev)
    vt = _dev_tensor(v, torch.int32, dev)
    k = int(ut.numel())
    if offsets_64bit is None:
        offsets_64bit = 2 * k > 0x7FFFFFFF
    wsb = ctypes.c_size_t()
    _check(lib().cc_csr_workspace_bytes(n, k, ctypes.byref(wsb)), "cc_csr_workspace_bytes")
    ws = torch.empty(max(int(wsb.value), 256), dtype=torch.uint8, device=dev)
    offsets = torch.empty(n + 1, dtype=torch.int64 if offsets_64bit else torch.int32, device=dev)
    adj = torch.empty(max(2 * k, 1), dtype=torch.int32, device=dev)
    m_dev = torch.zeros(1, dtype=torch.int64, device=dev)
    _check(lib().cc_build_csr(ctx.h, n, k, _ptr(ut), _ptr(vt), int(dedup), _ptr(ws), ws.numel(), _ptr(offsets),
                              int(offsets_64bit), _ptr(adj), _ptr(m_dev), _stream_handle(stream)),
           "cc_build_csr")
    m = int(m_dev.item())
    del ws
    return CSR(n, offsets, adj[:m])


class RenumberedCSR(CSR):
    """A device CSR of the graph with its vertices renumbered by decreasing
    degree (cc_build_csr_degree_order): orig_of[x] is the original id of
    vertex x, new_of its inverse (both int32[n] on the device).  n_active:
    rows n_active .. n-1 are empty (n when unknown)."""

    def __init__(self, n: int, offsets: torch.Tensor, adj: torch.Tensor, orig_of: torch.Tensor,
                 new_of: torch.Tensor, n_active: int | None = None):
        super().__init__(n, offsets, adj)
        self.orig_of = orig_of
        self.new_of = new_of
        self.n_active = n if n_active is None else int(n_active)


def build_csr_degree_order(ctx: Context, n: int, u, v, dedup: bool = True, offsets_64bit: bool | None = None,
                           stream=None) -> RenumberedCSR:
    """cc_build_csr_degree_order: the CSR of the pair list with vertices
    renumbered by decreasing degree (ties by id), and the permutation."""
    dev = ctx.torch_device
    ut = _dev_tensor(u, torch.int32, dev)
    vt = _dev_tensor(v, torch.int32, dev)
    k = int(ut.numel())
    if offsets_64bit is None:
        offsets_64bit = 2 * k > 0x7FFFFFFF
    wsb = ctypes.c_size_t()
    _check(lib().cc_csr_degree_order_workspace_bytes(n, k, ctypes.byref(wsb)), "cc_csr_degree_order_workspace_bytes")
    ws = torch.empty(max(int(wsb.value), 256), dtype=torch.uint8, device=dev)
    offsets = torch.empty(n + 1, dtype=torch.int64 if offsets_64bit else torch.int32, device=dev)
    adj = torch.empty(max(2 * k, 1), dtype=torch.int32, device=dev)
    m_dev = torch.zeros(1, dtype=torch.int64, device=dev)
    orig_of = torch.empty(n, dtype=torch.int32, device=dev)
    new_of = torch.empty(n, dtype=torch.int32, device=dev)
    _check(lib().cc_build_csr_degree_order(ctx.h, n, k, _ptr(ut), _ptr(vt), int(dedup), _ptr(ws), ws.numel(),
                                           _ptr(offsets), int(offsets_64bit), _ptr(adj), _ptr(m_dev), _ptr(orig_of),
                                           _ptr(new_of), _stream_handle(stream)),
           "cc_build_csr_degree_order")
    m = int(m_dev.item())
    del ws
    act = torch.zeros(1, dtype=torch.int64, device=dev)
    _check(lib().cc_csr_active_prefix(n, _ptr(offsets), int(offsets_64bit), _ptr(act), _stream_handle(stream)),
           "cc_csr_active_prefix")
    return RenumberedCSR(n, offsets, adj[:m], orig_of, new_of, int(act.item()))


def csr_active_prefix(g: CSR, stream=None) -> int:
    """cc_csr_active_prefix: the smallest x with rows x .. n-1 empty."""
    act = torch.zeros(1, dtype=torch.int64, device=g.offsets.device)
    _check(lib().cc_csr_active_prefix(g.n, _ptr(g.offsets), g.o64, _ptr(act), _stream_handle(stream)),
           "cc_csr_active_prefix")
    return int(act.item())


def connectivity_csr_mapped(ctx: Context, g: RenumberedCSR, variant: cc_variant | None = None,
                            labels: torch.Tensor | None = None, ncomp: torch.Tensor | None = None, stream=None):
    """cc_connectivity_csr_mapped on a renumbered CSR: labels (int32[n], in
    the original numbering: each vertex's smallest original id in its
    component) and the component count."""
    v = variant if variant is not None else default_variant()
    dev = ctx.torch_device
    if labels is None:
        labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    if ncomp is None:
        ncomp = torch.empty(1, dtype=torch.int64, device=dev)
    b = ctypes.c_size_t()
    _check(lib().cc_mapped_workspace_bytes(g.n, g.m, ctypes.byref(v), ctypes.byref(b)), "cc_mapped_workspace_bytes")
    ws = ctx.workspace(int(b.value))
    _check(lib().cc_connectivity_csr_mapped(ctx.h, g.n, g.n_active, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj),
                                            _ptr(g.orig_of), _ptr(g.new_of), ctypes.byref(v), _ptr(ws), ws.numel(),
                                            _ptr(labels), _ptr(ncomp), _stream_handle(stream)),
           "cc_connectivity_csr_mapped")
    return labels, ncomp


def validate_csr(ctx: Context, g: CSR, check_symmetric: bool = True, stream=None):
    """cc_validate_csr.  Returns (status, report dict): status CC_OK for a
    valid CSR, CC_EDEVICE when a check failed (report["failed"] holds the
    CSR_* bits).  Argument errors raise."""
    r = cc_csr_report()
    st = lib().cc_validate_csr(ctx.h, g.n, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj) if g.m else ctypes.c_void_p(0),
                               int(check_symmetric), ctypes.byref(r), _stream_handle(stream))
    if st not in (CC_OK, CC_EDEVICE) or (st == CC_EDEVICE and r.failed == 0):
        raise CCError(st, "cc_validate_csr")
    return st, r.as_dict()


def connectivity_csr(ctx: Context, g: CSR, variant: cc_variant | None = None, labels: torch.Tensor | None = None,
                     ncomp: torch.Tensor | None = None, stream=None):
    """cc_connectivity_csr.  Returns (labels int32[n], num_components int64[1]) on the device."""
    v = variant if variant is not None else default_variant()
    dev = ctx.torch_device
    if labels is None:
        labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    if ncomp is None:
        ncomp = torch.empty(1, dtype=torch.int64, device=dev)
    ws = ctx.workspace(workspace_bytes(g.n, g.m, v))
    _check(lib().cc_connectivity_csr(ctx.h, g.n, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj), ctypes.byref(v),
                                     _ptr(ws), ws.numel(), _ptr(labels), _ptr(ncomp), _stream_handle(stream)),
           "cc_connectivity_csr")
    return labels, ncomp


def noalloc_scratch_bytes() -> int:
    return int(lib().cc_noalloc_scratch_bytes())


def connectivity_csr_noalloc(ctx: Context, g: CSR, variant: cc_variant | None = None,
                             labels: torch.Tensor | None = None, ncomp: torch.Tensor | None = None, stream=None):
    """cc_connectivity_csr_noalloc: as connectivity_csr, with the library's
    fixed per-device workspace (pass labels/ncomp to allocate nothing here)."""
    v = variant if variant is not None else default_variant()
    dev = ctx.torch_device
    if labels is None:
        labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    if ncomp is None:
        ncomp = torch.empty(1, dtype=torch.int64, device=dev)
    _check(lib().cc_connectivity_csr_noalloc(ctx.h, g.n, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj),
                                             ctypes.byref(v), _ptr(labels), _ptr(ncomp), _stream_handle(stream)),
           "cc_connectivity_csr_noalloc")
    return labels, ncomp


def connectivity_coo(ctx: Context, n: int, u, v, variant: cc_variant | None = None,
                     labels: torch.Tensor | None = None, ncomp: torch.Tensor | None = None, stream=None):
    """cc_connectivity_coo on an undirected pair list (device or host int32
    arrays; host arrays are copied to the device first).  Returns (labels,
    num_components int64[1]) on the device."""
    var = variant if variant is not None else default_variant()
    dev = ctx.torch_device
    ut = _dev_tensor(u, torch.int32, dev)
    vt = _dev_tensor(v, torch.int32, dev)
    k = int(ut.numel())
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=dev)
    if ncomp is None:
        ncomp = torch.empty(1, dtype=torch.int64, device=dev)
    wsb = ctypes.c_size_t()
    _check(lib().cc_coo_workspace_bytes(n, k, ctypes.byref(var), ctypes.byref(wsb)), "cc_coo_workspace_bytes")
    ws = ctx.workspace(int(wsb.value))
    _check(lib().cc_connectivity_coo(ctx.h, n, k, _ptr(ut), _ptr(vt), ctypes.byref(var), _ptr(ws), ws.numel(),
                                     _ptr(labels), _ptr(ncomp), _stream_handle(stream)), "cc_connectivity_coo")
    return labels, ncomp


def spanning_forest_csr(ctx: Context, g: CSR, variant: cc_variant | None = None, stream=None):
    """cc_spanning_forest_csr.  Returns (labels int32[n], edges_u, edges_v,
    num_edges int64[1]); the first num_edges entries of edges_u/v are the forest."""
    v = variant if variant is not None else default_variant()
    dev = ctx.torch_device
    labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    eu = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    ev = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    ne = torch.zeros(1, dtype=torch.int64, device=dev)
    wsb = ctypes.c_size_t()
    _check(lib().cc_forest_workspace_bytes(g.n, g.m, ctypes.byref(v), ctypes.byref(wsb)), "cc_forest_workspace_bytes")
    ws = ctx.workspace(int(wsb.value))
    _check(lib().cc_spanning_forest_csr(ctx.h, g.n, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj), ctypes.byref(v),
                                        _ptr(ws), ws.numel(), _ptr(labels), _ptr(eu), _ptr(ev), _ptr(ne),
                                        _stream_handle(stream)), "cc_spanning_forest_csr")
    return labels, eu, ev, ne


def spanning_forest_csr_mapped(ctx: Context, g: RenumberedCSR, variant: cc_variant | None = None, stream=None):
    """cc_spanning_forest_csr_mapped.  Returns (labels int32[n], edges_u,
    edges_v, num_edges int64[1]) in the original numbering."""
    v = variant if variant is not None else default_variant()
    dev = ctx.torch_device
    labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    eu = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    ev = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    ne = torch.zeros(1, dtype=torch.int64, device=dev)
    wsb = ctypes.c_size_t()
    _check(lib().cc_forest_mapped_workspace_bytes(g.n, g.m, ctypes.byref(v), ctypes.byref(wsb)),
           "cc_forest_mapped_workspace_bytes")
    ws = ctx.workspace(int(wsb.value))
    _check(lib().cc_spanning_forest_csr_mapped(ctx.h, g.n, g.n_active, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj),
                                               _ptr(g.orig_of), _ptr(g.new_of), ctypes.byref(v), _ptr(ws),
                                               ws.numel(), _ptr(labels), _ptr(eu), _ptr(ev), _ptr(ne),
                                               _stream_handle(stream)), "cc_spanning_forest_csr_mapped")
    return labels, eu, ev, ne


def amsf_options(epsilon: float | None = None, light_fraction: float | None = None,
                 seed: int | None = None) -> cc_amsf_options:
    """cc_amsf_default_options with the given fields replaced."""
    o = cc_amsf_options()
    _check(lib().cc_amsf_default_options(ctypes.byref(o)), "cc_amsf_default_options")
    if epsilon is not None:
        o.epsilon = epsilon
    if light_fraction is not None:
        o.light_fraction = light_fraction
    if seed is not None:
        o.seed = seed
    return o


def amsf_csr(ctx: Context, g: CSR, weights, options: cc_amsf_options | None = None, stream=None):
    """cc_amsf_csr (Section 5.1).  weights: device float32 tensor of g.m
    entries, one per adjacency entry.  Returns (labels int32[n], edges_u,
    edges_v, edges_w, num_edges int64[1], weight float64[1]); the first
    num_edges entries of edges_u/v/w are the forest."""
    o = options if options is not None else amsf_options()
    dev = ctx.torch_device
    labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    eu = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    ev = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    ew = torch.empty(max(g.n, 1), dtype=torch.float32, device=dev)
    ne = torch.zeros(1, dtype=torch.int64, device=dev)
    tw = torch.zeros(1, dtype=torch.float64, device=dev)
    if weights.dtype != torch.float32 or weights.numel() != g.m:
        raise ValueError(f"weights must be float32 with {g.m} entries")
    wsb = ctypes.c_size_t()
    _check(lib().cc_amsf_workspace_bytes(g.n, g.m, ctypes.byref(o), ctypes.byref(wsb)), "cc_amsf_workspace_bytes")
    ws = ctx.workspace(int(wsb.value))
    wp = _ptr(weights) if g.m > 0 else None
    _check(lib().cc_amsf_csr(ctx.h, g.n, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj), wp, ctypes.byref(o), _ptr(ws),
                             ws.numel(), _ptr(labels), _ptr(eu), _ptr(ev), _ptr(ew), _ptr(ne), _ptr(tw),
                             _stream_handle(stream)), "cc_amsf_csr")
    return labels, eu, ev, ew, ne, tw


def amsf_csr_mapped(ctx: Context, g: RenumberedCSR, weights, options: cc_amsf_options | None = None, stream=None):
    """cc_amsf_csr_mapped: as amsf_csr on a renumbered CSR (weights per
    adjacency entry of that CSR), edges and labels in the original numbering."""
    o = options if options is not None else amsf_options()
    dev = ctx.torch_device
    labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    eu = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    ev = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    ew = torch.empty(max(g.n, 1), dtype=torch.float32, device=dev)
    ne = torch.zeros(1, dtype=torch.int64, device=dev)
    tw = torch.zeros(1, dtype=torch.float64, device=dev)
    if weights.dtype != torch.float32 or weights.numel() != g.m:
        raise ValueError(f"weights must be float32 with {g.m} entries")
    wsb = ctypes.c_size_t()
    _check(lib().cc_amsf_mapped_workspace_bytes(g.n, g.m, ctypes.byref(o), ctypes.byref(wsb)),
           "cc_amsf_mapped_workspace_bytes")
    ws = ctx.workspace(int(wsb.value))
    wp = _ptr(weights) if g.m > 0 else None
    _check(lib().cc_amsf_csr_mapped(ctx.h, g.n, g.n_active, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj), _ptr(g.orig_of),
                                    _ptr(g.new_of), wp, ctypes.byref(o), _ptr(ws), ws.numel(), _ptr(labels),
                                    _ptr(eu), _ptr(ev), _ptr(ew), _ptr(ne), _ptr(tw), _stream_handle(stream)),
           "cc_amsf_csr_mapped")
    return labels, eu, ev, ew, ne, tw


def sample_csr(ctx: Context, g: CSR, variant: cc_variant, stream=None):
    """cc_sample_csr: the sampled partial labelling and the chosen frequent label."""
    dev = ctx.torch_device
    labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    ws = ctx.workspace(workspace_bytes(g.n, g.m, variant))
    lm = ctypes.c_int32(-2)
    _check(lib().cc_sample_csr(ctx.h, g.n, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj), ctypes.byref(variant),
                               _ptr(ws), ws.numel(), _ptr(labels), ctypes.byref(lm), _stream_handle(stream)),
           "cc_sample_csr")
    return labels, int(lm.value)


class Stream:
    """cc_stream: device-resident batch-incremental connectivity state."""

    def __init__(self, ctx: Context, n: int, variant: cc_variant | None = None):
        self.ctx = ctx
        self.n = n
        self.h = ctypes.c_void_p()
        vp = ctypes.byref(variant) if variant is not None else None
        _check(lib().cc_stream_create(ctx.h, n, vp, ctypes.byref(self.h)), "cc_stream_create")

    def close(self):
        if self.h:
            lib().cc_stream_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_csr(self, g: CSR, variant: cc_variant, stream=None):
        ws = self.ctx.workspace(workspace_bytes(g.n, g.m, variant))
        _check(lib().cc_stream_init_csr(self.h, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj), _ptr(ws), ws.numel(),
                                        _stream_handle(stream)), "cc_stream_init_csr")

    def insert(self, u, v, stream=None):
        """Insert(u[i], v[i]); host arrays are copied to the device first."""
        dev = self.ctx.torch_device
        u = _dev_tensor(u, torch.int32, dev)
        v = _dev_tensor(v, torch.int32, dev)
        if u.numel() != v.numel():
            raise ValueError("u and v differ in length")
        _check(lib().cc_insert_batch(self.h, int(u.numel()), _ptr(u), _ptr(v), _stream_handle(stream)),
               "cc_insert_batch")

    def query(self, a, b, out: torch.Tensor | None = None, stream=None):
        """IsConnected(a[i], b[i]) as a device uint8 tensor."""
        dev = self.ctx.torch_device
        a = _dev_tensor(a, torch.int32, dev)
        b = _dev_tensor(b, torch.int32, dev)
        if a.numel() != b.numel():
            raise ValueError("a and b differ in length")
        if out is None:
            out = torch.empty(int(a.numel()), dtype=torch.uint8, device=dev)
        elif out.dtype != torch.uint8 or out.numel() < a.numel():
            raise ValueError("out must be a uint8 tensor with one byte per pair")
        _check(lib().cc_query_batch(self.h, int(a.numel()), _ptr(a), _ptr(b), _ptr(out), _stream_handle(stream)),
               "cc_query_batch")
        return out

    def process(self, kind, u, v, out: torch.Tensor | None = None, stream=None):
        """cc_process_batch: one mixed batch; kind[i] == 0 inserts (u[i], v[i]),
        any other kind asks IsConnected(u[i], v[i]).  Returns the device
        uint8 answers (0 for inserts)."""
        dev = self.ctx.torch_device
        kd = _dev_tensor(kind, torch.uint8, dev)
        u = _dev_tensor(u, torch.int32, dev)
        v = _dev_tensor(v, torch.int32, dev)
        if not (kd.numel() == u.numel() == v.numel()):
            raise ValueError("kind, u and v differ in length")
        if out is None:
            out = torch.empty(int(u.numel()), dtype=torch.uint8, device=dev)
        elif out.dtype != torch.uint8 or out.numel() < u.numel():
            raise ValueError("out must be a uint8 tensor with one byte per operation")
        _check(lib().cc_process_batch(self.h, int(u.numel()), _ptr(kd), _ptr(u), _ptr(v), _ptr(out),
                                      _stream_handle(stream)), "cc_process_batch")
        return out

    @property
    def type(self) -> int:
        """Streaming type of the finish: 1, 2 or 3 (Section 3.4)."""
        return int(lib().cc_stream_type(self.h))

    def labels(self, stream=None):
        dev = self.ctx.torch_device
        lab = torch.empty(self.n, dtype=torch.int32, device=dev)
        nc = torch.empty(1, dtype=torch.int64, device=dev)
        _check(lib().cc_stream_labels(self.h, _ptr(lab), _ptr(nc), _stream_handle(stream)), "cc_stream_labels")
        return lab, nc

    def sync_status(self):
        _check(lib().cc_stream_sync_status(self.h), "cc_stream_sync_status")


# ---- serving loop --------------------------------------------------------------

def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else ctypes.c_void_p(0)


class Server:
    """cc_server: continuous batching of insert/query requests (host arrays)."""

    def __init__(self, ctx: Context, n: int, variant: cc_variant | None = None, budget_bytes: int = 1 << 30,
                 num_streams: int = 4, max_inflight: int = 64):
        self.ctx = ctx
        self.n = n
        self.h = ctypes.c_void_p()
        vp = ctypes.byref(variant) if variant is not None else None
        _check(lib().cc_server_create(ctx.h, n, vp, budget_bytes, num_streams, max_inflight, ctypes.byref(self.h)),
               "cc_server_create")
        self._keep = []

    def close(self):
        if self.h:
            lib().cc_server_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clock(self) -> float:
        return lib().cc_server_clock(self.h)

    def insert(self, u, v, arrival: float = -1.0) -> int:
        import numpy as np
        u = np.ascontiguousarray(u, np.int32)
        v = np.ascontiguousarray(v, np.int32)
        self._keep += [u, v]          # the server reads them until the request completes
        rid = ctypes.c_int64()
        _check(lib().cc_server_submit_insert(self.h, u.size, _np_ptr(u), _np_ptr(v), arrival, ctypes.byref(rid)),
               "cc_server_submit_insert")
        return rid.value

    def query(self, a, b, arrival: float = -1.0):
        """Returns (request id, output array filled when the request completes)."""
        import numpy as np
        a = np.ascontiguousarray(a, np.int32)
        b = np.ascontiguousarray(b, np.int32)
        out = np.zeros(a.size, np.uint8)
        self._keep += [a, b, out]
        rid = ctypes.c_int64()
        _check(lib().cc_server_submit_query(self.h, a.size, _np_ptr(a), _np_ptr(b), _np_ptr(out), arrival,
                                            ctypes.byref(rid)), "cc_server_submit_query")
        return rid.value, out

    def poll(self, wait_all: bool = False):
        _check(lib().cc_server_poll(self.h, int(wait_all)), "cc_server_poll")

    def info(self, rid: int):
        done = ctypes.c_int()
        lat = ctypes.c_double()
        _check(lib().cc_server_request_info(self.h, rid, ctypes.byref(done), ctypes.byref(lat)),
               "cc_server_request_info")
        return bool(done.value), lat.value

    def run_trace(self, types, arrivals, starts, lens, a, b, out=None):
        """Real-time replay; returns (query answers aligned with a/b, latencies).
        a, b and out may be pinned (e.g. numpy views of pinned torch tensors)."""
        import numpy as np
        types = np.ascontiguousarray(types, np.int32)
        arrivals = np.ascontiguousarray(arrivals, np.float64)
        starts = np.ascontiguousarray(starts, np.int64)
        lens = np.ascontiguousarray(lens, np.int64)
        a = np.ascontiguousarray(a, np.int32)
        b = np.ascontiguousarray(b, np.int32)
        if out is None:
            out = np.zeros(a.size, np.uint8)
        lat = np.zeros(types.size, np.float64)
        _check(lib().cc_server_run_trace(self.h, types.size, _np_ptr(types), _np_ptr(arrivals), _np_ptr(starts),
                                         _np_ptr(lens), _np_ptr(a), _np_ptr(b), _np_ptr(out), _np_ptr(lat)),
               "cc_server_run_trace")
        return out, lat

    def labels(self):
        dev = self.ctx.torch_device
        lab = torch.empty(self.n, dtype=torch.int32, device=dev)
        nc = torch.empty(1, dtype=torch.int64, device=dev)
        _check(lib().cc_server_labels(self.h, _ptr(lab), _ptr(nc), _stream_handle()), "cc_server_labels")
        return lab, nc

    def pool_used(self) -> int:
        return int(lib().cc_server_pool_used(self.h))

    @property
    def stamped(self) -> bool:
        """True when queries overlap later inserts (UF-Async + FindNaive)."""
        return bool(lib().cc_server_stamped(self.h))

    def event_count(self) -> int:
        return int(lib().cc_server_event_count(self.h))


# ---- selector ---------------------------------------------------------------------

def mlp_param_count(K: int) -> int:
    return int(lib().cc_mlp_param_count(K))


def mlp_forward(params_bf16: torch.Tensor, K: int, X: torch.Tensor, cache: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
    """params_bf16: int16/uint16-typed device tensor of BF16 bit patterns; X: [B,16] float32."""
    B = int(X.shape[0])
    Y = torch.empty(B, K, dtype=torch.float32, device=X.device)
    _check(lib().cc_mlp_forward(_ptr(params_bf16), K, B, _ptr(X), _ptr(Y), _ptr(cache), _stream_handle(stream)),
           "cc_mlp_forward")
    return Y


def mlp_backward(params_bf16, K, X, cache, Y, T, stream=None):
    B = int(X.shape[0])
    dev = X.device
    grads = torch.empty(mlp_param_count(K), dtype=torch.float32, device=dev)
    scratch = torch.empty(4 * B * 64, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    _check(lib().cc_mlp_backward(_ptr(params_bf16), K, B, _ptr(X), _ptr(cache), _ptr(Y), _ptr(T), _ptr(grads),
                                 _ptr(scratch), _ptr(loss), _stream_handle(stream)), "cc_mlp_backward")
    return grads, loss


def mlp_adam(master, params_bf16, grads, m1, m2, lr, beta1, beta2, eps, step, stream=None):
    _check(lib().cc_mlp_adam(_ptr(master), _ptr(params_bf16), _ptr(grads), _ptr(m1), _ptr(m2), master.numel(), lr,
                             beta1, beta2, eps, step, _stream_handle(stream)), "cc_mlp_adam")


def mlp_pack_bf16(src: torch.Tensor, dst: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if dst is None:
        dst = torch.empty(src.numel(), dtype=torch.int16, device=src.device)
    _check(lib().cc_mlp_pack_bf16(_ptr(src), _ptr(dst), src.numel(), _stream_handle(stream)), "cc_mlp_pack_bf16")
    return dst


def graph_features(ctx: Context, g: CSR, stream=None):
    """The 16 selector features (host list of floats)."""
    ws = ctx.workspace(workspace_bytes(g.n, g.m, default_variant()))
    f = (ctypes.c_float * 16)()
    _check(lib().cc_graph_features(ctx.h, g.n, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj), _ptr(ws), ws.numel(), f,
                                   _stream_handle(stream)), "cc_graph_features")
    return [float(x) for x in f]


class Selector:
    """A trained model bound to its arms: the ctypes arrays are built once so
    that a call costs one C call (features, forward pass and argmin on the
    device, then the chosen arm)."""

    def __init__(self, ctx: Context, params_bf16: torch.Tensor | None, arms, norm, gate=None):
        """gate: (min_vertices, arm) -- smaller graphs run that arm without the
        model (cc_ctx_set_selector_gate); None leaves the gate off."""
        self.ctx = ctx
        gv, ga = gate if gate is not None else (0, -1)
        _check(lib().cc_ctx_set_selector_gate(ctx.h, int(gv), int(ga)), "cc_ctx_set_selector_gate")
        self.params = params_bf16
        self.arms = list(arms) if arms is not None else []
        self.K = len(self.arms) if params_bf16 is not None else 0
        if params_bf16 is not None and params_bf16.numel() != mlp_param_count(self.K):
            raise ValueError(f"the model has {params_bf16.numel()} parameters; {len(self.arms)} arms need "
                             f"{mlp_param_count(self.K)}")
        self._arr = (cc_variant * max(self.K, 1))(*self.arms[:self.K]) if self.K else None
        self._norm = (ctypes.c_float * 32)(*[float(x) for x in norm]) if norm is not None else None
        self._need = {}
        self._args = {}
        self._feat = (ctypes.c_float * 16)()
        self._chosen = ctypes.c_int32(-2)

    def _ws(self, g: CSR):
        key = (g.n, g.m)
        if key not in self._need:
            need = workspace_bytes(g.n, g.m, default_variant())
            for a in self.arms[:self.K]:
                need = max(need, workspace_bytes(g.n, g.m, a))
            self._need[key] = need
        return self.ctx.workspace(self._need[key])

    def connectivity(self, g: CSR, labels: torch.Tensor, ncomp: torch.Tensor, stream=None):
        """cc_connectivity_auto: returns the chosen arm index (-1 = default).
        The marshalled arguments are cached per (graph, outputs, stream), so
        a repeated call costs one C call."""
        hs = _stream_handle(stream)
        key = (id(g), g.offsets.data_ptr(), g.adj.data_ptr(), labels.data_ptr(), ncomp.data_ptr(), hs.value)
        args = self._args.get(key)
        if args is None:
            ws = self._ws(g)
            if labels.numel() < g.n or ncomp.numel() < 1:
                raise ValueError("labels needs n entries and ncomp one")
            args = (self.ctx.h, g.n, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj), _ptr(self.params), self.K, self._arr,
                    self._norm, _ptr(ws), ws.numel(), _ptr(labels), _ptr(ncomp), ctypes.byref(self._chosen),
                    self._feat, hs, (g, labels, ncomp, ws))
            self._args = {key: args}    # keep one entry: the tensors it references stay alive
        _check(lib().cc_connectivity_auto(*args[:-1]), "cc_connectivity_auto")
        return self._chosen.value

    def features(self):
        """Features of the last call."""
        return [float(x) for x in self._feat]

    def select(self, g: CSR, stream=None):
        """cc_select_variant: (variant, arm index or -1, features) without running it."""
        ws = self._ws(g)
        out = cc_variant()
        _check(lib().cc_select_variant(self.ctx.h, g.n, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj),
                                       _ptr(self.params), self.K, self._arr, self._norm, _ptr(ws), ws.numel(),
                                       ctypes.byref(out), ctypes.byref(self._chosen), self._feat,
                                       _stream_handle(stream)), "cc_select_variant")
        return out, self._chosen.value, self.features()


def connectivity_auto(ctx: Context, g: CSR, params_bf16: torch.Tensor | None, arms, norm, labels=None, ncomp=None,
                      stream=None):
    """cc_connectivity_auto: returns (labels, ncomp, chosen arm index, features)."""
    dev = ctx.torch_device
    if labels is None:
        labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    if ncomp is None:
        ncomp = torch.empty(1, dtype=torch.int64, device=dev)
    sel = Selector(ctx, params_bf16, arms, norm)
    chosen = sel.connectivity(g, labels, ncomp, stream)
    return labels, ncomp, chosen, sel.features()


def select_variant(ctx: Context, g: CSR, params_bf16: torch.Tensor | None, arms, norm, stream=None):
    """cc_select_variant: (chosen variant, arm index or -1, features) without running it."""
    return Selector(ctx, params_bf16, arms, norm).select(g, stream)


# ---- calibration -------------------------------------------------------------

def calib_copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    nbytes = min(src.numel() * src.element_size(), dst.numel() * dst.element_size())
    _check(lib().cc_calib_copy(_ptr(src), _ptr(dst), nbytes - nbytes % 16, _stream_handle(stream)), "cc_calib_copy")


def calib_edges(g: CSR, vals: torch.Tensor | None = None, out: torch.Tensor | None = None, stream=None):
    """MapEdges (vals None) or GatherEdges over a device CSR; returns out (n int32)."""
    if out is None:
        out = torch.empty(g.n, dtype=torch.int32, device=g.adj.device)
    wsb = ctypes.c_size_t()
    _check(lib().cc_calib_workspace_bytes(g.m, ctypes.byref(wsb)), "cc_calib_workspace_bytes")
    ws = torch.empty(int(wsb.value), dtype=torch.uint8, device=g.adj.device)
    _check(lib().cc_calib_edges(g.n, g.m, _ptr(g.offsets), g.o64, _ptr(g.adj), _ptr(vals), _ptr(out), _ptr(ws),
                                ws.numel(), _stream_handle(stream)), "cc_calib_edges")
    return out


# ---- the variant space ---------------------------------------------------------

def all_finishes():
    """The 20 finish methods: 9 Rem-CAS, 4 Async, SV, 6 root-based Liu-Tarjan."""
    out = []
    for sp in (SPLICE_SPLIT_ONE, SPLICE_HALVE_ONE, SPLICE_ATOMIC):
        for fd in (FIND_NAIVE, FIND_ATOMIC_SPLIT, FIND_ATOMIC_HALVE):
            out.append(dict(finish=FIN_UF_REM_CAS, splice=sp, find=fd))
    for fd in (FIND_NAIVE, FIND_ATOMIC_SPLIT, FIND_ATOMIC_HALVE, FIND_COMPRESS):
        out.append(dict(finish=FIN_UF_ASYNC, find=fd, splice=0))
    out.append(dict(finish=FIN_SV, find=0, splice=0))
    for r in (LT_CRSA, LT_PRSA, LT_PRS, LT_CRFA, LT_PRFA, LT_PRF):
        out.append(dict(finish=FIN_LT, lt_rules=r, find=0, splice=0))
    return out


def extra_finishes():
    """The 19 further finishes of Section 3.3 and the appendix: UF-Early and
    UF-Hooks with each find, label propagation, and the 10 non-root-based
    Liu-Tarjan variants."""
    out = []
    for fin in (FIN_UF_EARLY, FIN_UF_HOOKS):
        for fd in (FIND_NAIVE, FIND_ATOMIC_SPLIT, FIND_ATOMIC_HALVE, FIND_COMPRESS):
            out.append(dict(finish=fin, find=fd, splice=0))
    out.append(dict(finish=FIN_LP, find=0, splice=0))
    for r in LT_NONROOT.values():
        out.append(dict(finish=FIN_LT, lt_rules=r, find=0, splice=0))
    return out


def all_variants(seed: int = 0x5EED, extended: bool = False):
    """Every sampling x finish combination: the 80 of the main table
    (4 samplers x 20 finishes); with extended=True 76 more follow them (the
    4 samplers x extra_finishes()), so indices below 80 never change."""
    base = default_variant(seed=seed)
    out = []
    for s in (SAMPLE_NONE, SAMPLE_KOUT, SAMPLE_BFS, SAMPLE_LDD):
        for f in all_finishes():
            out.append(base.copy(sample=s, **f))
    if extended:
        for s in (SAMPLE_NONE, SAMPLE_KOUT, SAMPLE_BFS, SAMPLE_LDD):
            for f in extra_finishes():
                out.append(base.copy(sample=s, **f))
    return out
