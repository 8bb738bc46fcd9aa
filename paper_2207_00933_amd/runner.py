"""Buffer management and call sequencing around libsqc for whole workloads.

Nothing here computes: it allocates device buffers with PyTorch, uploads the
variant probabilities, and calls the C entry points in order (attribute every
subcircuit once, then recurse / search / contract).  The product path fails
loudly when the HIP library or a GPU is missing.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np
import torch

from . import sqc

_TORCH_DTYPE = {sqc.F64: torch.float64, sqc.F32: torch.float32}


def _bytes_tensor(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Session:
    """One context on one device with a caller-owned workspace."""

    def __init__(self, device: int = 0, workspace_bytes: int = 64 << 20):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the reconstruction runs only on the HIP library")
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = sqc.ctx_create(device, self.stream.cuda_stream)
        self.ws = None
        self.ensure_workspace(workspace_bytes)

    def ensure_workspace(self, nbytes: int) -> None:
        if self.ws is not None and self.ws.numel() >= nbytes:
            return
        self.ws = _bytes_tensor(nbytes, self.device)
        sqc.ctx_set_workspace(self.ctx, self.ws)

    def close(self) -> None:
        if self.ctx:
            torch.cuda.synchronize(self.device)
            sqc.ctx_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Circuit:
    """A compute graph with its variants resident on the device."""

    def __init__(self, session: Session, graph: sqc.Graph,
                 variants: Sequence[np.ndarray], var_prec: int = sqc.F64):
        self.s = session
        self.g = graph
        self.var_prec = var_prec
        dt = _TORCH_DTYPE[var_prec]
        self.var = [torch.from_numpy(np.ascontiguousarray(v)).to(dt).to(session.device)
                    for v in variants]
        self.att: List[sqc.Tensor] = []
        self.att_buf: List[torch.Tensor] = []

    @classmethod
    def from_cut_circuit(cls, session: Session, cc, variants, var_prec: int = sqc.F64):
        return cls(session, sqc.Graph.from_cut_circuit(cc), variants, var_prec)

    def attribute(self, out_prec: int = sqc.F64, merged: bool = False) -> List[sqc.Tensor]:
        """Attribute every subcircuit (subcircuits that fit the on-chip stage
        share one launch); merged=True writes the merged layout of a
        full-output recursion instead (sqc_attribute_all_merged)."""
        if len(self.att_buf) != self.g.n_sub or self.att[0].prec != out_prec:
            self.att_buf = [_bytes_tensor(sqc.attribute_bytes(self.g, i, out_prec), self.s.device)
                            for i in range(self.g.n_sub)]
        fn = sqc.attribute_all_merged if merged else sqc.attribute_all
        self.att = fn(self.s.ctx, self.g, self.var, self.var_prec, self.att_buf, out_prec)
        return self.att

    def attributed_numpy(self, i: int) -> np.ndarray:
        """Attributed tensor i as [2^d][4^c] float64 (host copy)."""
        t = self.att[i]
        n = (1 << t.n_bits) << (2 * t.n_labels)
        dt = _TORCH_DTYPE[t.prec]
        x = self.att_buf[i][: n * (8 if t.prec == sqc.F64 else 4)].view(dt).double().cpu().numpy()
        if t.layout == sqc.LAYOUT_MERGED:  # [4^c][2^d]
            return x.reshape(1 << (2 * t.n_labels), 1 << t.n_bits).T.copy()
        return x.reshape(1 << t.n_bits, 1 << (2 * t.n_labels))


class Recursion:
    """Output buffers for sqc_recurse at a given largest bin count."""

    def __init__(self, circ: Circuit, max_bits: int, bins_prec: int, top_r: int):
        s = circ.s
        self.c = circ
        self.bins_prec = bins_prec
        self.top_r = top_r
        self.bins = torch.empty(1 << max_bits, dtype=_TORCH_DTYPE[bins_prec], device=s.device)
        self._ws = {}
        self.top = torch.empty(2 * sqc.MAX_TOPR, dtype=torch.float64, device=s.device)
        self.sum = torch.empty(1, dtype=torch.float64, device=s.device)

    def run(self, prec: int, M: int, scope=None) -> List[sqc.Masks]:
        c = self.c
        # reserve workspace for the masks this call will use (remembered per
        # scope, M and precision: planning is host work)
        key = (prec, M, None if scope is None else tuple(sqc.masks_array(scope)[i].as_tuple()
                                                         for i in range(len(scope))),
               tuple((t.prec, t.n_bits, t.n_labels, t.layout) for t in c.att))
        need = self._ws.get(key)
        if need is None:
            masks = sqc.assign_bins(c.g.n_data, scope, M)
            need = sqc.recurse_workspace_bytes(c.att, c.g, masks, prec)
            if need == 0:
                raise RuntimeError(sqc.lib().sqc_last_error(None).decode())
            self._ws[key] = need
        c.s.ensure_workspace(need)
        return sqc.recurse(c.s.ctx, c.att, c.g, scope, M, self.top_r, prec, self.bins,
                           self.bins_prec, self.top, self.sum)

    def top_list(self):
        t = self.top.cpu().numpy()
        vals = t[0:2 * self.top_r:2]
        idx = t[1:2 * self.top_r:2].view(np.uint64)
        return vals, idx


def active_bits(masks: Sequence[sqc.Masks]) -> int:
    return sum(bin(m.active).count("1") for m in masks)


class Server:
    """The serving engine with a device workspace of its own.  Output buffers
    of a request are the caller's and must stay alive until it is done; the
    request structs (with their scope arrays) are kept here until then."""

    def __init__(self, device: int = 0, n_slots: int = 4, workspace_bytes: int = 256 << 20,
                 max_batch: int = 128):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the serving engine runs only on the HIP library")
        self.device = torch.device("cuda", device)
        self.ws = _bytes_tensor(workspace_bytes, self.device)
        self.srv = sqc.serve_create(device, n_slots, self.ws)
        sqc.serve_set_max_batch(self.srv, max_batch)
        self.graphs = {}
        self._live = {}

    def register(self, circ: Circuit) -> int:
        # the attributed tensors were written on the session's stream
        torch.cuda.synchronize(self.device)
        cid = sqc.serve_register(self.srv, circ.att, circ.g)
        self.graphs[cid] = circ.g
        return cid

    def request(self, cid: int, scope, M: int, top_r: int, prec: int, bins, bins_prec: int,
                topr, bsum, masks_out: bool = False) -> sqc.Request:
        n_sub = self.graphs[cid].n_sub
        mo = (sqc.Masks * n_sub)() if masks_out else None
        r = sqc.make_request(cid, n_sub, scope, M, top_r, prec, bins, bins_prec, topr, bsum, mo)
        r._masks = mo
        return r

    def footprint(self, req: sqc.Request) -> int:
        return sqc.serve_footprint(self.srv, req)

    def submit(self, req: sqc.Request) -> int:
        t = sqc.serve_submit(self.srv, req)
        self._live[t] = req
        return t

    def submit_many(self, reqs: Sequence[sqc.Request]) -> List[int]:
        ts = sqc.serve_submit_many(self.srv, reqs)
        for t, r in zip(ts, reqs):
            self._live[t] = r
        return ts

    def poll(self, ticket: int) -> int:
        st = sqc.serve_poll(self.srv, ticket)
        if st == sqc.DONE:
            self._live.pop(ticket, None)
        return st

    def wait(self, ticket: int) -> None:
        sqc.serve_wait(self.srv, ticket)
        self._live.pop(ticket, None)

    def completed(self, cap: int = 256) -> List[int]:
        done = sqc.serve_completed(self.srv, cap)
        for t in done:
            self._live.pop(t, None)
        return done

    def stats(self) -> sqc.ServeStats:
        return sqc.serve_get_stats(self.srv)

    def close(self) -> None:
        if self.srv:
            sqc.serve_destroy(self.srv)
            self.srv = 0
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
