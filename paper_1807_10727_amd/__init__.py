"""LocalContraction connected components on one AMD Instinct MI355X (gfx950).

The work runs in the HIP library ``libcc.so`` (C ABI in ``include/cc.h``); this package
only marshals arguments.  PyTorch provides device memory (the caller's edge tensors, the
workspace, the label tensor) and the stream.

    from paper_1807_10727_amd import Solver
    s = Solver(n, src, dst, seed=1)        # src/dst: int32 or int64 CUDA tensors
    rounds = s.run()
    labels = s.labels()                    # int32 (or int64) CUDA tensor [n]
"""
from __future__ import annotations

from . import _cc
from ._cc import (cc_batch_create, cc_batch_destroy, cc_batch_get_config, cc_batch_run, cc_batch_set_config,
                  cc_batch_set_workspace, cc_batch_split, cc_batch_workspace_size)
from ._cc import (cc_server_cancel, cc_server_pause, cc_server_create, cc_server_destroy, cc_server_info, cc_server_poll,
                  cc_server_submit, cc_server_wait)
from ._cc import (CC_CANONICAL, CC_DONE, CC_EDGES_PACKED_U64, CC_EDGES_SOA_I32, CC_EDGES_SOA_I64, CC_OK,
                  CC_EAGER, CC_EXPLICIT_PRIO, CC_MERGE_TO_LARGE, CC_ONE_HOP, CC_PROFILE, CC_RECORD_ROUNDS,
                  CC_ROUND0_DIRECT,
                  CC_ROUND0_TILED, CC_TREE, CCError, cc_debug_round_arrays, cc_load_state, cc_save_state,
                  cc_set_explicit_priorities, cc_set_merge_to_large, cc_get_tuning, cc_set_tuning,
                  cc_contract_round, cc_create, cc_destroy, cc_get_finished, cc_get_round_sorted, cc_get_round_stats, cc_kernel_family_names, cc_kernel_times,
                  cc_labels, cc_last_error, cc_reset, cc_round_edges, cc_round_parents, cc_run, cc_set_finish, cc_set_profile_mask,
                  cc_set_workspace, cc_version, cc_workspace_size, TUNING_KNOBS)

__all__ = ["Solver", "Batch", "Server", "solve", "CCError", "CC_CANONICAL", "CC_EAGER", "CC_EXPLICIT_PRIO",
           "CC_MERGE_TO_LARGE",
           "CC_ONE_HOP", "CC_PROFILE", "CC_RECORD_ROUNDS", "CC_ROUND0_DIRECT", "CC_ROUND0_TILED", "CC_TREE",
           "cc_version"]


def _torch():
    import torch
    return torch


class Solver:
    """One graph's solve behind the C ABI.  The edge tensors are borrowed (kept referenced)
    until close(); the workspace is a torch uint8 tensor on the same device."""

    def __init__(self, n: int, src, dst=None, seed: int = 0, max_rounds: int = 0, flags: int = 0,
                 stream=None, layout: int | None = None, finish_edges: int = 0):
        torch = _torch()
        if not src.is_cuda:
            raise ValueError("edge tensors must be device tensors")
        if layout is None:
            if dst is None:
                layout = CC_EDGES_PACKED_U64
            elif src.dtype == torch.int32:
                layout = CC_EDGES_SOA_I32
            elif src.dtype == torch.int64:
                layout = CC_EDGES_SOA_I64
            else:
                raise ValueError("unsupported edge dtype %s" % src.dtype)
        if dst is not None and (dst.dtype != src.dtype or dst.shape != src.shape):
            raise ValueError("src and dst must have the same dtype and shape")
        if not src.is_contiguous() or (dst is not None and not dst.is_contiguous()):
            raise ValueError("edge tensors must be contiguous")
        self.n = int(n)
        self.m = int(src.shape[0])
        self.layout = layout
        self.device = src.device
        self._src, self._dst = src, dst
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = cc_create(self.n, self.m, layout, src.data_ptr(), dst.data_ptr() if dst is not None else 0,
                             seed=seed, max_rounds=max_rounds, flags=flags, stream=self.stream.cuda_stream)
        self.ws_bytes = cc_workspace_size(self.ctx)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        cc_set_workspace(self.ctx, self.ws.data_ptr(), self.ws_bytes)
        if finish_edges:
            cc_set_finish(self.ctx, finish_edges)

    def set_tuning(self, round0: int = 0, blocks_per_cu: int = 0, round0_key_sets: int = 1, scatter_waves: int = 0,
                   row_pairs: int = 0, relabel_pairs: int = 0, row_generation: int = 0, round0_sort: int = 0,
                   tail: int = 0, radix_form: int = 0) -> None:
        """Tuning knobs (include/cc.h, cc_tuning); resets the solve.  A tiled round 0 needs a
        workspace sized for it: the one this object allocated when the context chose it."""
        cc_set_tuning(self.ctx, round0, blocks_per_cu, round0_key_sets, scatter_waves, row_pairs, relabel_pairs,
                      row_generation, round0_sort, tail, radix_form)

    @property
    def tuning(self) -> dict:
        return cc_get_tuning(self.ctx)

    def set_finish(self, max_edges: int) -> None:
        """Union-find finish once a round leaves at most max_edges edges (0: off)."""
        cc_set_finish(self.ctx, max_edges)

    @property
    def finished(self) -> bool:
        """Whether the current solve ended with the union-find finish."""
        return cc_get_finished(self.ctx)

    @property
    def label_dtype(self):
        torch = _torch()
        return torch.int64 if self.layout == CC_EDGES_SOA_I64 else torch.int32

    def run(self) -> int:
        return cc_run(self.ctx)

    def contract_round(self):
        return cc_contract_round(self.ctx)

    def labels(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self.n, dtype=self.label_dtype, device=self.device)
        cc_labels(self.ctx, out.data_ptr() if self.n else 1)
        return out

    def parents(self, r: int = -1):
        """Parents of round r (default: the most recent one), by name (-1 for names that were
        not nodes), and the round's node count.  Earlier rounds need CC_RECORD_ROUNDS."""
        torch = _torch()
        out = torch.empty(max(self.n, 1), dtype=torch.int32, device=self.device)
        k = cc_round_parents(self.ctx, r, out.data_ptr())
        return out[:self.n], k

    def minima(self):
        """One-hop and two-hop minima of the most recent round by name (uint32 values in
        int32 tensors; -1 = 0xFFFFFFFF for names that were not nodes)."""
        torch = _torch()
        m1 = torch.empty(max(self.n, 1), dtype=torch.int32, device=self.device)
        l2 = torch.empty(max(self.n, 1), dtype=torch.int32, device=self.device)
        cc_debug_round_arrays(self.ctx, m1.data_ptr(), l2.data_ptr())
        return m1[:self.n], l2[:self.n]

    def set_priorities(self, r: int, table) -> None:
        """Explicit priorities from round r on (CC_EXPLICIT_PRIO): an int32 device tensor of
        n values, a permutation of 0 .. n-1, kept referenced while the context lives."""
        if not table.is_cuda or table.numel() < self.n or not table.is_contiguous():
            raise ValueError("the table must be a contiguous device tensor of n entries")
        self._tables = getattr(self, "_tables", {})
        self._tables[int(r)] = table
        cc_set_explicit_priorities(self.ctx, r, table.data_ptr())

    def set_merge_to_large(self, alphas) -> None:
        """MergeToLarge parameters of phases 0, 1, ... (CC_MERGE_TO_LARGE)."""
        cc_set_merge_to_large(self.ctx, alphas)

    def save_state(self) -> bytes:
        return cc_save_state(self.ctx)

    def load_state(self, data: bytes) -> None:
        cc_load_state(self.ctx, data)

    def edges(self):
        """Edges of the graph the last round left, by name: an int64 tensor of
        (a << 32) | b with a < b, one entry per distinct edge, in no particular order."""
        torch = _torch()
        m = cc_round_edges(self.ctx, 0, 0)            # the count only
        out = torch.empty(max(m, 1), dtype=torch.int64, device=self.device)
        k = cc_round_edges(self.ctx, out.data_ptr(), out.numel())
        return out[:k]

    def stats(self, rounds: int):
        return [cc_get_round_stats(self.ctx, r) for r in range(rounds)]

    def sorted_keys(self, rounds: int):
        """For each round, the keys its duplicate drop processed (include/cc.h,
        cc_round_stats.m_sorted)."""
        return [cc_get_round_sorted(self.ctx, r) for r in range(rounds)]

    def rounds_in_graph(self, rounds: int):
        """For each round, whether it ran inside a captured tail (include/cc.h, cc_run)."""
        return [bool(cc_get_round_stats(self.ctx, r, True)[-1]) for r in range(rounds)]

    def reset(self, seed: int) -> None:
        cc_reset(self.ctx, seed)

    def kernel_times(self):
        return cc_kernel_times(self.ctx)

    def profile_families(self, names=None) -> None:
        """Time only these kernel families under CC_PROFILE (None: all)."""
        cc_set_profile_mask(self.ctx, names)

    def close(self) -> None:
        if self.ctx:
            cc_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(n: int, src, dst=None, seed: int = 0, flags: int = 0, max_rounds: int = 0, finish_edges: int = 0):
    """Full solve: returns (labels tensor, rounds, per-round stats)."""
    with Solver(n, src, dst, seed=seed, flags=flags, max_rounds=max_rounds, finish_edges=finish_edges) as s:
        rounds = s.run()
        lab = s.labels()
        st = s.stats(rounds)
        _torch().cuda.current_stream(s.device).synchronize()
        return lab, rounds, st


class Batch:
    """Many independent graphs solved together (cc_batch_*).  Graph g has vertices
    0 .. n_g-1 and records src[i], dst[i] (int32 local ids, device tensors) for i in
    [edge_off[g], edge_off[g+1]); seeds[g] is its priority seed.  Labels come back as one
    int32 tensor with graph g's labels at [vtx_off[g], vtx_off[g+1])."""

    def __init__(self, vtx_off, edge_off, seeds, src, dst, stream=None, ws_fill=None, **config):
        torch = _torch()
        import numpy as np
        self.voff = np.ascontiguousarray(vtx_off, dtype=np.int64)
        self.eoff = np.ascontiguousarray(edge_off, dtype=np.int64)
        self.G = int(self.voff.shape[0] - 1)
        self.n_total = int(self.voff[-1])
        self.device = src.device
        if src.dtype != torch.int32 or dst.dtype != torch.int32:
            raise ValueError("batched records are int32 local ids")
        self._src, self._dst = src, dst
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.b = cc_batch_create(self.voff, self.eoff, seeds, src.data_ptr(), dst.data_ptr(),
                                 stream=self.stream.cuda_stream)
        self.ws_bytes = cc_batch_workspace_size(self.b)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        if ws_fill is not None:   # a workspace that starts with these bytes (tests)
            self.ws.fill_(int(ws_fill))
        cc_batch_set_workspace(self.b, self.ws.data_ptr(), self.ws_bytes)
        if config:
            cc_batch_set_config(self.b, **config)
        self.labels_buf = torch.empty(max(self.n_total, 1), dtype=torch.int32, device=self.device)

    def configure(self, **config):
        cc_batch_set_config(self.b, **config)

    @property
    def config(self):
        return cc_batch_get_config(self.b)

    def split(self):
        return cc_batch_split(self.b)

    def run(self, with_rounds: bool = True):
        import numpy as np
        rounds = np.zeros(max(self.G, 1), dtype=np.int32) if with_rounds else None
        cc_batch_run(self.b, self.labels_buf.data_ptr(), rounds)
        return self.labels_buf[:self.n_total], (rounds[:self.G] if with_rounds else None)

    def close(self):
        if self.b:
            cc_batch_destroy(self.b)
            self.b = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over the C ABI (cc_server_*).  The arena is a torch uint8
    tensor of `budget` bytes; submitted tensors are kept referenced until their request
    completes."""

    def __init__(self, budget: int, device="cuda:0", **config):
        torch = _torch()
        self.device = torch.device(device)
        self.arena = torch.empty(budget, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        self.srv = cc_server_create(self.arena.data_ptr(), budget, **config)
        self._held = {}

    def submit(self, n: int, src, dst, seed: int, labels=None, layout: int | None = None):
        """Returns (request id, labels tensor).  src/dst: int32 (or int64) device tensors."""
        torch = _torch()
        if layout is None:
            layout = CC_EDGES_SOA_I32 if src.dtype == torch.int32 else CC_EDGES_SOA_I64
        if labels is None:
            labels = torch.empty(max(n, 1), dtype=torch.int64 if layout == CC_EDGES_SOA_I64 else torch.int32,
                                 device=self.device)
        rid = cc_server_submit(self.srv, n, int(src.shape[0]), layout, src.data_ptr(),
                               dst.data_ptr() if dst is not None else 0, seed, labels.data_ptr())
        self._held[rid] = (src, dst, labels)
        return rid, labels[:n]

    def _release(self, results):
        for r in results:
            self._held.pop(r["id"], None)
        return results

    def poll(self):
        return self._release(cc_server_poll(self.srv))

    def wait(self, timeout_s: float = 1.0):
        return self._release(cc_server_wait(self.srv, timeout_s))

    def drain(self, timeout_s: float = 600.0):
        """Wait for every submitted request; returns their results."""
        import time
        out = []
        t_end = time.time() + timeout_s
        while self._held and time.time() < t_end:
            out += self.wait(0.5)
        return out

    def pause(self, paused: bool = True) -> None:
        """Admit no new request while paused (requests in flight continue)."""
        cc_server_pause(self.srv, paused)

    def cancel(self, rid: int):
        cc_server_cancel(self.srv, rid)

    def info(self):
        return cc_server_info(self.srv)

    def close(self):
        if self.srv:
            cc_server_destroy(self.srv)
            self.srv = None
            self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
