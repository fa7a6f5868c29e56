"""ctypes binding of libcc.so (include/cc.h): argument marshalling only.

Every step of a solve runs in the HIP library; this module passes pointers and sizes.
Importing it fails loudly when libcc.so has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libcc.so is not built (run __graft_entry__.build() or "
                      "python paper_1807_10727_amd/build.py); there is no fallback path")

_lib = ctypes.CDLL(LIB_PATH)

CC_OK, CC_DONE = 0, 1
CC_E_ARG, CC_E_INPUT, CC_E_NOMEM, CC_E_HIP, CC_E_STATE, CC_E_BUDGET = -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "CC_OK", 1: "CC_DONE", -1: "CC_E_ARG", -2: "CC_E_INPUT", -3: "CC_E_NOMEM", -4: "CC_E_HIP",
                -5: "CC_E_STATE", -6: "CC_E_BUDGET"}

CC_EDGES_SOA_I32, CC_EDGES_SOA_I64, CC_EDGES_PACKED_U64 = 0, 1, 2
CC_CANONICAL = 1 << 0
CC_PROFILE = 1 << 1
CC_ROUND0_DIRECT = 1 << 2
CC_ROUND0_TILED = 1 << 3
CC_EAGER = 1 << 4
CC_TREE = 1 << 5
CC_ONE_HOP = 1 << 6
CC_EXPLICIT_PRIO = 1 << 7
CC_RECORD_ROUNDS = 1 << 8
CC_MERGE_TO_LARGE = 1 << 9


class cc_graph_desc(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("n_edges", ctypes.c_int64), ("layout", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p)]


class cc_options(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("max_rounds", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("stream", ctypes.c_void_p)]


class cc_round_stats(ctypes.Structure):
    _fields_ = [("round", ctypes.c_int32), ("in_graph", ctypes.c_int32), ("n_active", ctypes.c_int64),
                ("m_in", ctypes.c_int64), ("m_survive", ctypes.c_int64), ("m_out", ctypes.c_int64),
                ("n_finalised", ctypes.c_int64), ("m_sorted", ctypes.c_int64)]

    def as_tuple(self):
        return (self.round, self.n_active, self.m_in, self.m_survive, self.m_out, self.n_finalised)


TUNING_KNOBS = ("round0", "blocks_per_cu", "round0_key_sets", "scatter_waves", "row_pairs", "relabel_pairs",
                "row_generation", "round0_sort", "tail", "radix_form")


class cc_tuning(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in TUNING_KNOBS]

    def as_dict(self):
        return {k: getattr(self, k) for k in TUNING_KNOBS}


class cc_batch_config(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("small_variant", ctypes.c_int32),
                ("small_threads", ctypes.c_int32), ("small_blocks_per_cu", ctypes.c_int32),
                ("rounds_per_graph", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("radix_form", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class cc_server_config(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("small_variant", ctypes.c_int32), ("small_threads", ctypes.c_int32),
                ("small_blocks_per_cu", ctypes.c_int32), ("max_small_per_launch", ctypes.c_int32),
                ("small_launches", ctypes.c_int32), ("cohort_max", ctypes.c_int32),
                ("cohort_max_vertices", ctypes.c_int32)]


class cc_request_result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("small_path", ctypes.c_int32), ("cohort", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class cc_server_info_t(ctypes.Structure):
    _fields_ = [("now", ctypes.c_double), ("pending", ctypes.c_int64), ("active", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_int64), ("peak_bytes", ctypes.c_int64), ("small_launches", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_ctx_p = ctypes.c_void_p
_sig = {
    "cc_create": (ctypes.c_int32, [ctypes.POINTER(cc_graph_desc), ctypes.POINTER(cc_options),
                                   ctypes.POINTER(_ctx_p)]),
    "cc_workspace_size": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(ctypes.c_size_t)]),
    "cc_set_workspace": (ctypes.c_int32, [_ctx_p, ctypes.c_void_p, ctypes.c_size_t]),
    "cc_reset": (ctypes.c_int32, [_ctx_p, ctypes.c_uint64]),
    "cc_set_tuning": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(cc_tuning)]),
    "cc_get_tuning": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(cc_tuning)]),
    "cc_contract_round": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(cc_round_stats)]),
    "cc_run": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(ctypes.c_int32)]),
    "cc_labels": (ctypes.c_int32, [_ctx_p, ctypes.c_void_p]),
    "cc_round_parents": (ctypes.c_int32, [_ctx_p, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "cc_debug_round_arrays": (ctypes.c_int32, [_ctx_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cc_set_explicit_priorities": (ctypes.c_int32, [_ctx_p, ctypes.c_int32, ctypes.c_void_p]),
    "cc_set_merge_to_large": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
    "cc_save_state": (ctypes.c_int32, [_ctx_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "cc_load_state": (ctypes.c_int32, [_ctx_p, ctypes.c_void_p, ctypes.c_size_t]),
    "cc_round_edges": (ctypes.c_int32, [_ctx_p, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "cc_get_round_stats": (ctypes.c_int32, [_ctx_p, ctypes.c_int32, ctypes.POINTER(cc_round_stats)]),
    "cc_kernel_family_count": (ctypes.c_int32, []),
    "cc_set_profile_mask": (ctypes.c_int32, [_ctx_p, ctypes.c_uint64]),
    "cc_set_finish": (ctypes.c_int32, [_ctx_p, ctypes.c_int64]),
    "cc_get_finished": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(ctypes.c_int32)]),
    "cc_kernel_family_name": (ctypes.c_char_p, [ctypes.c_int32]),
    "cc_kernel_times": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.c_int32]),
    "cc_destroy": (ctypes.c_int32, [_ctx_p]),
    "cc_last_error": (ctypes.c_char_p, [_ctx_p]),
    "cc_version": (ctypes.c_char_p, []),
    "cc_batch_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(cc_options), ctypes.POINTER(_ctx_p)]),
    "cc_batch_workspace_size": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(ctypes.c_size_t)]),
    "cc_batch_set_workspace": (ctypes.c_int32, [_ctx_p, ctypes.c_void_p, ctypes.c_size_t]),
    "cc_batch_set_config": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(cc_batch_config)]),
    "cc_batch_get_config": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(cc_batch_config)]),
    "cc_batch_run": (ctypes.c_int32, [_ctx_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cc_batch_split": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]),
    "cc_batch_destroy": (ctypes.c_int32, [_ctx_p]),
    "cc_batch_last_error": (ctypes.c_char_p, [_ctx_p]),
    "cc_server_create": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(cc_server_config),
                                          ctypes.POINTER(_ctx_p)]),
    "cc_server_submit": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(cc_graph_desc), ctypes.c_uint64, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "cc_server_poll": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(cc_request_result), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]),
    "cc_server_wait": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(cc_request_result), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.c_double]),
    "cc_server_pause": (ctypes.c_int32, [_ctx_p, ctypes.c_int32]),
    "cc_server_cancel": (ctypes.c_int32, [_ctx_p, ctypes.c_uint64]),
    "cc_server_info": (ctypes.c_int32, [_ctx_p, ctypes.POINTER(cc_server_info_t)]),
    "cc_server_destroy": (ctypes.c_int32, [_ctx_p]),
    "cc_server_last_error": (ctypes.c_char_p, [_ctx_p]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class CCError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


def _check(ctx, status: int) -> int:
    if status < 0:
        msg = _lib.cc_last_error(ctx) if ctx else b""
        raise CCError(status, (msg or b"").decode())
    return status


# ---- same names as the C ABI -----------------------------------------------------------

def cc_create(n_vertices: int, n_edges: int, layout: int, src_ptr: int, dst_ptr: int, seed: int = 0,
              max_rounds: int = 0, flags: int = 0, stream: int = 0):
    g = cc_graph_desc(n_vertices, n_edges, layout, 0, src_ptr or None, dst_ptr or None)
    o = cc_options(seed & 0xFFFFFFFFFFFFFFFF, max_rounds, flags, stream or None)
    ctx = _ctx_p()
    _check(None, _lib.cc_create(ctypes.byref(g), ctypes.byref(o), ctypes.byref(ctx)))
    return ctx


def cc_workspace_size(ctx) -> int:
    n = ctypes.c_size_t()
    _check(ctx, _lib.cc_workspace_size(ctx, ctypes.byref(n)))
    return int(n.value)


def cc_set_workspace(ctx, ptr: int, nbytes: int) -> None:
    _check(ctx, _lib.cc_set_workspace(ctx, ptr, nbytes))


def cc_reset(ctx, seed: int) -> None:
    _check(ctx, _lib.cc_reset(ctx, seed & 0xFFFFFFFFFFFFFFFF))


def cc_set_tuning(ctx, round0: int = 0, blocks_per_cu: int = 0, round0_key_sets: int = 1, scatter_waves: int = 0,
                  row_pairs: int = 0, relabel_pairs: int = 0, row_generation: int = 0, round0_sort: int = 0,
                  tail: int = 0, radix_form: int = 0) -> None:
    """Knobs of include/cc.h's cc_tuning; 0 keeps a knob's default (round0: the current form)."""
    t = cc_tuning(int(round0), int(blocks_per_cu), int(round0_key_sets), int(scatter_waves), int(row_pairs),
                  int(relabel_pairs), int(row_generation), int(round0_sort), int(tail), int(radix_form))
    _check(ctx, _lib.cc_set_tuning(ctx, ctypes.byref(t)))


def cc_get_tuning(ctx) -> dict:
    t = cc_tuning()
    _check(ctx, _lib.cc_get_tuning(ctx, ctypes.byref(t)))
    return t.as_dict()


def cc_contract_round(ctx):
    """Returns (status, stats tuple or None); status is CC_OK or CC_DONE."""
    s = cc_round_stats()
    st = _check(ctx, _lib.cc_contract_round(ctx, ctypes.byref(s)))
    return st, (s.as_tuple() if st == CC_OK else None)


def cc_run(ctx) -> int:
    r = ctypes.c_int32()
    _check(ctx, _lib.cc_run(ctx, ctypes.byref(r)))
    return int(r.value)


def cc_labels(ctx, ptr: int) -> None:
    _check(ctx, _lib.cc_labels(ctx, ptr))


def cc_round_parents(ctx, r: int, ptr: int) -> int:
    """Parents of round r (r < 0: the most recent one) by name into the device buffer at ptr
    (int32[n_vertices]); returns the round's node count."""
    n = ctypes.c_int64()
    _check(ctx, _lib.cc_round_parents(ctx, int(r), ptr, ctypes.byref(n)))
    return int(n.value)


def cc_debug_round_arrays(ctx, m1_ptr: int, l_ptr: int) -> None:
    """One-hop and two-hop minima of the most recent round by name (uint32[n_vertices] each)."""
    _check(ctx, _lib.cc_debug_round_arrays(ctx, m1_ptr, l_ptr))


def cc_set_explicit_priorities(ctx, r: int, ptr: int) -> None:
    """Round r and later use the priority table at ptr (uint32[n_vertices], a permutation)."""
    _check(ctx, _lib.cc_set_explicit_priorities(ctx, int(r), ptr))


def cc_set_merge_to_large(ctx, alphas) -> None:
    """MergeToLarge parameters of phases 0, 1, ... (the last one repeats)."""
    a = (ctypes.c_int64 * len(alphas))(*[int(x) for x in alphas])
    _check(ctx, _lib.cc_set_merge_to_large(ctx, a, len(alphas)))


def cc_save_state(ctx) -> bytes:
    """The context's round checkpoint as bytes (two calls: size, then the copy)."""
    n = ctypes.c_size_t(0)
    _check(ctx, _lib.cc_save_state(ctx, None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(ctx, _lib.cc_save_state(ctx, buf, ctypes.byref(n)))
    return buf.raw[:n.value]


def cc_load_state(ctx, data: bytes) -> None:
    buf = ctypes.create_string_buffer(data, len(data))
    _check(ctx, _lib.cc_load_state(ctx, buf, len(data)))


def cc_round_edges(ctx, ptr: int, cap: int) -> int:
    """Edges of the graph the last round left, by name, into the device buffer at ptr
    (uint64[cap]); returns their number (include/cc.h)."""
    n = ctypes.c_int64()
    _check(ctx, _lib.cc_round_edges(ctx, ptr, int(cap), ctypes.byref(n)))
    return int(n.value)


def cc_get_round_stats(ctx, r: int, with_graph_flag: bool = False):
    s = cc_round_stats()
    _check(ctx, _lib.cc_get_round_stats(ctx, r, ctypes.byref(s)))
    return s.as_tuple() + ((s.in_graph,) if with_graph_flag else ())


def cc_set_finish(ctx, max_edges: int) -> None:
    _check(ctx, _lib.cc_set_finish(ctx, int(max_edges)))


def cc_get_finished(ctx) -> bool:
    f = ctypes.c_int32()
    _check(ctx, _lib.cc_get_finished(ctx, ctypes.byref(f)))
    return bool(f.value)


def cc_get_round_sorted(ctx, r: int) -> int:
    """Keys the sort of round r processed (cc_round_stats.m_sorted)."""
    s = cc_round_stats()
    _check(ctx, _lib.cc_get_round_stats(ctx, r, ctypes.byref(s)))
    return int(s.m_sorted)


def cc_kernel_family_names():
    return [_lib.cc_kernel_family_name(i).decode() for i in range(_lib.cc_kernel_family_count())]


def cc_set_profile_mask(ctx, names) -> None:
    """Time only the named kernel families under CC_PROFILE (None: all)."""
    if names is None:
        mask = (1 << 64) - 1
    else:
        fams = cc_kernel_family_names()
        mask = 0
        for n in names:
            mask |= 1 << fams.index(n)
    _check(ctx, _lib.cc_set_profile_mask(ctx, mask))


def cc_kernel_times(ctx):
    k = _lib.cc_kernel_family_count()
    ms = (ctypes.c_double * k)()
    ln = (ctypes.c_int64 * k)()
    _check(ctx, _lib.cc_kernel_times(ctx, ms, ln, k))
    return {name: (ms[i], ln[i]) for i, name in enumerate(cc_kernel_family_names())}


def cc_destroy(ctx) -> None:
    if ctx:
        _lib.cc_destroy(ctx)


def cc_last_error(ctx) -> str:
    return (_lib.cc_last_error(ctx) or b"").decode()


def cc_version() -> str:
    return _lib.cc_version().decode()


# ---- batched solve ---------------------------------------------------------------------

def _bcheck(b, status: int) -> int:
    if status < 0:
        msg = _lib.cc_batch_last_error(b) if b else b""
        raise CCError(status, (msg or b"").decode())
    return status


def cc_batch_create(vtx_off, edge_off, seeds, src_ptr: int, dst_ptr: int, flags: int = 0, stream: int = 0):
    import numpy as np
    voff = np.ascontiguousarray(vtx_off, dtype=np.int64)
    eoff = np.ascontiguousarray(edge_off, dtype=np.int64)
    sd = np.ascontiguousarray(seeds, dtype=np.uint64)
    G = int(voff.shape[0] - 1)
    o = cc_options(0, 0, flags, stream or None)
    b = _ctx_p()
    _bcheck(None, _lib.cc_batch_create(G, voff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       eoff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       sd.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), src_ptr or None,
                                       dst_ptr or None, ctypes.byref(o), ctypes.byref(b)))
    return b


def cc_batch_workspace_size(b) -> int:
    n = ctypes.c_size_t()
    _bcheck(b, _lib.cc_batch_workspace_size(b, ctypes.byref(n)))
    return int(n.value)


def cc_batch_set_workspace(b, ptr: int, nbytes: int) -> None:
    _bcheck(b, _lib.cc_batch_set_workspace(b, ptr, nbytes))


def cc_batch_set_config(b, **kw) -> None:
    c = cc_batch_config()
    _bcheck(b, _lib.cc_batch_get_config(b, ctypes.byref(c)))
    for k, v in kw.items():
        setattr(c, k, int(v))
    _bcheck(b, _lib.cc_batch_set_config(b, ctypes.byref(c)))


def cc_batch_get_config(b) -> dict:
    c = cc_batch_config()
    _bcheck(b, _lib.cc_batch_get_config(b, ctypes.byref(c)))
    return c.as_dict()


def cc_batch_run(b, labels_ptr: int, rounds=None) -> None:
    """rounds: optional host int32 numpy array [G] receiving per-graph round counts."""
    rp = rounds.ctypes.data_as(ctypes.c_void_p) if rounds is not None else None
    _bcheck(b, _lib.cc_batch_run(b, labels_ptr or None, rp))


def cc_batch_split(b):
    ns = ctypes.c_int32()
    um = ctypes.c_int64()
    _bcheck(b, _lib.cc_batch_split(b, ctypes.byref(ns), ctypes.byref(um)))
    return int(ns.value), int(um.value)


def cc_batch_destroy(b) -> None:
    if b:
        _lib.cc_batch_destroy(b)


def cc_batch_last_error(b) -> str:
    return (_lib.cc_batch_last_error(b) or b"").decode()


# ---- serving ---------------------------------------------------------------------------

def _scheck(srv, status: int) -> int:
    if status < 0:
        msg = _lib.cc_server_last_error(srv) if srv else b""
        raise CCError(status, (msg or b"").decode())
    return status


def cc_server_create(arena_ptr: int, budget: int, n_slots: int = 4, small_variant: int = 1, small_threads: int = 256,
                     small_blocks_per_cu: int = 2, max_small_per_launch: int = 1024, small_launches: int = 2,
                     cohort_max: int = 0, cohort_max_vertices: int = 0):
    c = cc_server_config(n_slots, small_variant, small_threads, small_blocks_per_cu, max_small_per_launch,
                         small_launches, cohort_max, cohort_max_vertices)
    srv = _ctx_p()
    _scheck(None, _lib.cc_server_create(arena_ptr, budget, ctypes.byref(c), ctypes.byref(srv)))
    return srv


def cc_server_submit(srv, n_vertices: int, n_edges: int, layout: int, src_ptr: int, dst_ptr: int, seed: int,
                     labels_ptr: int) -> int:
    g = cc_graph_desc(n_vertices, n_edges, layout, 0, src_ptr or None, dst_ptr or None)
    rid = ctypes.c_uint64()
    _scheck(srv, _lib.cc_server_submit(srv, ctypes.byref(g), seed & 0xFFFFFFFFFFFFFFFF, labels_ptr or None,
                                       ctypes.byref(rid)))
    return int(rid.value)


def cc_server_poll(srv, cap: int = 256):
    out = (cc_request_result * cap)()
    n = ctypes.c_int32()
    _scheck(srv, _lib.cc_server_poll(srv, out, cap, ctypes.byref(n)))
    return [out[i].as_dict() for i in range(n.value)]


def cc_server_wait(srv, timeout_s: float = 1.0, cap: int = 256):
    out = (cc_request_result * cap)()
    n = ctypes.c_int32()
    _scheck(srv, _lib.cc_server_wait(srv, out, cap, ctypes.byref(n), timeout_s))
    return [out[i].as_dict() for i in range(n.value)]


def cc_server_cancel(srv, rid: int) -> None:
    _scheck(srv, _lib.cc_server_cancel(srv, rid))


def cc_server_pause(srv, paused: bool) -> None:
    _scheck(srv, _lib.cc_server_pause(srv, 1 if paused else 0))


def cc_server_info(srv) -> dict:
    i = cc_server_info_t()
    _scheck(srv, _lib.cc_server_info(srv, ctypes.byref(i)))
    return i.as_dict()


def cc_server_destroy(srv) -> None:
    if srv:
        _lib.cc_server_destroy(srv)


def cc_server_last_error(srv) -> str:
    return (_lib.cc_server_last_error(srv) or b"").decode()
