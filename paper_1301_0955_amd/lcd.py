"""Python binding of the C ABI in include/lcd.h (liblcd.so).

Argument marshalling only: every step of the sweep and of the readout runs
in the library's HIP kernels.  PyTorch supplies device memory and the
current stream.  There is no fallback: if the built library is missing,
importing or calling this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblcd.so")

LCD_OK, LCD_EINVAL, LCD_ENOMEM, LCD_EDEVICE, LCD_EAGAIN, LCD_ECAPACITY, LCD_ESTATE, LCD_ECANCELED = range(8)
LCD_MEM_HOST, LCD_MEM_DEVICE = 0, 1
LCD_PERSISTENT, LCD_PER_SCALE_LOOP = 0, 1
LCD_OUT_FULL, LCD_OUT_DELTA = 0, 1

_STATUS = {0: "LCD_OK", 1: "LCD_EINVAL", 2: "LCD_ENOMEM", 3: "LCD_EDEVICE", 4: "LCD_EAGAIN",
           5: "LCD_ECAPACITY", 6: "LCD_ESTATE", 7: "LCD_ECANCELED"}


class LcdError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__("%s: %s (%s)" % (where, msg, _STATUS.get(status, status)))
        self.status = status


class lcd_params(ctypes.Structure):
    _fields_ = [("k_prune", ctypes.c_uint32), ("mode", ctypes.c_int32),
                ("lds_capacity", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("pool_hint", ctypes.c_int64), ("watchdog_ms", ctypes.c_int32),
                ("spill_mode", ctypes.c_int32), ("team_capacity", ctypes.c_int32),
                ("team_waves", ctypes.c_int32), ("grow_calls", ctypes.c_int32),
                ("queue_min_entries", ctypes.c_int32), ("output_mode", ctypes.c_int32)]


class lcd_tier_stats(ctypes.Structure):
    _fields_ = [("rows_gathered", ctypes.c_int64), ("row_entries", ctypes.c_int64),
                ("entries_created", ctypes.c_int64), ("members_written", ctypes.c_int64),
                ("sets_finished", ctypes.c_int64), ("entries_scanned", ctypes.c_int64),
                ("move_rows", ctypes.c_int64), ("move_row_entries", ctypes.c_int64),
                ("seed_rows", ctypes.c_int64), ("seed_row_entries", ctypes.c_int64),
                ("entries_committed", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lcd_sweep_stats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("ms_main", ctypes.c_double),
                ("ms_spill", ctypes.c_double), ("n_spilled", ctypes.c_int64),
                ("n_spilled_big", ctypes.c_int64), ("pool_used", ctypes.c_int64),
                ("reruns", ctypes.c_int32), ("lds_capacity", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("launches", ctypes.c_int32), ("tiers", ctypes.c_int32),
                ("tier", lcd_tier_stats * 4), ("ms_tier", ctypes.c_double * 4),
                ("tier_kind", ctypes.c_int32 * 4), ("tier_capacity", ctypes.c_int32 * 4)]

    def as_dict(self):
        arrays = ("tier", "ms_tier", "tier_kind", "tier_capacity")
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in arrays}
        d["tier"] = [t.as_dict() for t in self.tier]
        for k in arrays[1:]:
            d[k] = list(getattr(self, k))
        return d


class lcd_tune_report(ctypes.Structure):
    _fields_ = [("best", lcd_params), ("ms_best", ctypes.c_double), ("n_tried", ctypes.c_int32),
                ("sample_stride", ctypes.c_int32), ("full_checked", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("ms", ctypes.c_double * 16), ("tried", lcd_params * 16)]


def _params_dict(p: lcd_params) -> dict:
    return {k: getattr(p, k) for k, _ in lcd_params._fields_}


class lcd_query_info(ctypes.Structure):
    _fields_ = [("n_members", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("k_in", ctypes.c_int64), ("vol", ctypes.c_int64), ("f", ctypes.c_double),
                ("ctr", ctypes.c_uint64 * 4), ("t_submit_ns", ctypes.c_int64),
                ("t_start_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64),
                ("lane", ctypes.c_int32), ("pad", ctypes.c_int32)]


class lcd_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("requeued", ctypes.c_int64), ("pending", ctypes.c_int64),
                ("in_flight", ctypes.c_int64), ("mem_held", ctypes.c_int64),
                ("forwarded", ctypes.c_int64), ("spill_batches", ctypes.c_int64),
                ("lanes", ctypes.c_int32), ("spill_lanes", ctypes.c_int32),
                ("max_slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("max_lanes_busy", ctypes.c_int32), ("spill_tables", ctypes.c_int32 * 2),
                ("pad", ctypes.c_int32), ("cancelled", ctypes.c_int64), ("routed", ctypes.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("spill_tables", "pad")}
        d["spill_tables"] = list(self.spill_tables)
        return d


_lib = None
P = ctypes.c_void_p


def library() -> ctypes.CDLL:
    """The loaded liblcd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblcd.so is not built (run paper_1301_0955_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    sig = {
        "lcd_params_default": (None, [ctypes.POINTER(lcd_params)]),
        "lcd_graph_upload": (st, [ctypes.c_int32, ctypes.c_int64, P, P, P, ctypes.c_int32, P,
                                  ctypes.POINTER(P)]),
        "lcd_graph_info": (st, [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
        "lcd_graph_free": (st, [P]),
        "lcd_graph_upload_batch": (st, [ctypes.c_int32, P, P, P, P, P, ctypes.c_int32, P,
                                        ctypes.POINTER(P)]),
        "lcd_graph_batch_info": (st, [P, ctypes.POINTER(ctypes.c_int32), P]),
        "lcd_sweep_merge": (st, [P, P, ctypes.c_int32, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.POINTER(lcd_params), P, ctypes.POINTER(P)]),
        "lcd_result_merged_into": (st, [P, ctypes.c_int32, P]),
        "lcd_seeds": (st, [P, ctypes.c_int32, P, ctypes.c_int32, P, P, ctypes.POINTER(ctypes.c_int32)]),
        "lcd_sweep_batch": (st, [P, P, ctypes.c_int32, P, P, P, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.POINTER(lcd_params), P, ctypes.POINTER(P)]),
        "lcd_sweep": (st, [P, P, ctypes.c_int32, P, P, ctypes.c_int32, ctypes.c_int32,
                           ctypes.POINTER(lcd_params), P, ctypes.POINTER(P)]),
        "lcd_result_shape": (st, [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
        "lcd_result_sizes": (st, [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
        "lcd_result_membership": (st, [P, ctypes.c_int32, P, P, P, P, P, ctypes.c_int32, P]),
        "lcd_result_overlap": (st, [P, ctypes.c_int32, P, P, ctypes.c_int32, P]),
        "lcd_result_delta_sizes": (st, [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64)]),
        "lcd_result_delta": (st, [P, ctypes.c_int32, P, P, P, P, ctypes.c_int32, P]),
        "lcd_result_counters": (st, [P, P, P, ctypes.c_int32, P]),
        "lcd_result_stats": (st, [P, ctypes.POINTER(lcd_sweep_stats)]),
        "lcd_result_sets": (st, [P, P, ctypes.c_int32, P, P, P, ctypes.c_int64,
                                 ctypes.POINTER(ctypes.c_int64), P, P, P, P]),
        "lcd_result_free": (st, [P]),
        "lcd_result_rerun": (st, [P, P]),
        "lcd_log_device": (st, [P, P, ctypes.c_int64, P]),
        "lcd_device_info": (st, [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int64), ctypes.c_char_p, ctypes.c_int32]),
        "lcd_server_create": (st, [P, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(lcd_params),
                                   ctypes.POINTER(P)]),
        "lcd_server_submit": (st, [P, P, ctypes.c_int32, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_uint64)]),
        "lcd_server_poll": (st, [P, ctypes.c_uint64, P, ctypes.c_int32,
                                 ctypes.POINTER(lcd_query_info)]),
        "lcd_server_wait": (st, [P, ctypes.c_uint64, ctypes.c_int32]),
        "lcd_server_cancel": (st, [P, ctypes.c_uint64]),
        "lcd_server_get_stats": (st, [P, ctypes.POINTER(lcd_server_stats)]),
        "lcd_server_destroy": (st, [P]),
        "lcd_tune": (st, [P, P, ctypes.c_int32, P, P, ctypes.c_int32, ctypes.c_int32,
                          ctypes.POINTER(lcd_params), P, ctypes.POINTER(lcd_tune_report)]),
        "lcd_graph_untune": (st, [P]),
        "lcd_cover_nmi": (st, [ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int32, P, P,
                               ctypes.POINTER(ctypes.c_double), P]),
        "lcd_result_nmi": (st, [P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), P]),
        "lcd_result_nmi_successive": (st, [P, ctypes.c_int32, P, P]),
        "lcd_result_nmi_cover": (st, [P, ctypes.c_int32, ctypes.c_int32, P, P,
                                      ctypes.POINTER(ctypes.c_double), P]),
        "lcd_sweep_into": (st, [P, P, ctypes.c_int32, P, P, ctypes.c_int32, ctypes.c_int64,
                                ctypes.POINTER(lcd_params), P, P, P, P, P, P, P, ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_int64), P]),
        "lcd_last_error": (ctypes.c_char_p, []),
        "lcd_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int, where: str):
    if status != LCD_OK:
        msg = library().lcd_last_error().decode(errors="replace")
        raise LcdError(status, where, msg)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(a, dtype) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(device="cuda", dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to("cuda")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# Thin wrappers with the C names
# ---------------------------------------------------------------------------

def lcd_version() -> str:
    return library().lcd_version().decode()


def lcd_device_info() -> dict:
    cu = ctypes.c_int32()
    lc = ctypes.c_int64()
    lb = ctypes.c_int64()
    arch = ctypes.create_string_buffer(64)
    _check(library().lcd_device_info(ctypes.byref(cu), ctypes.byref(lc), ctypes.byref(lb), arch, 64),
           "lcd_device_info")
    return dict(compute_units=cu.value, lds_per_cu=lc.value, lds_per_block=lb.value,
                arch=arch.value.decode())


def lcd_log_device(x: torch.Tensor) -> torch.Tensor:
    """L(x) on the device for integer x in [1, 2^53) (int64 tensor)."""
    x = _dev(x, torch.int64)
    out = torch.empty(x.shape, dtype=torch.float64, device="cuda")
    _check(library().lcd_log_device(_ptr(x), _ptr(out), x.numel(), _stream()), "lcd_log_device")
    return out


class Graph:
    """A graph resident on the GPU (lcd_graph_upload)."""

    def __init__(self, n: int, row_ptr, col, w=None):
        self.n = int(n)
        rp = _dev(row_ptr, torch.int32)
        cl = _dev(col, torch.int32)
        ww = None if w is None else _dev(w, torch.uint8)
        h = P()
        _check(library().lcd_graph_upload(self.n, int(cl.numel()), _ptr(rp), _ptr(cl), _ptr(ww),
                                          LCD_MEM_DEVICE, _stream(), ctypes.byref(h)),
               "lcd_graph_upload")
        self._h = h

    @classmethod
    def from_host(cls, n, row_ptr, col, w=None):
        """Upload from host numpy arrays (the library validates and copies)."""
        self = cls.__new__(cls)
        self.n = int(n)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        ww = None if w is None else np.ascontiguousarray(w, dtype=np.uint8)
        h = P()
        _check(library().lcd_graph_upload(
            self.n, int(cl.size), rp.ctypes.data_as(P), cl.ctypes.data_as(P),
            None if ww is None else ww.ctypes.data_as(P), LCD_MEM_HOST, _stream(), ctypes.byref(h)),
            "lcd_graph_upload")
        self._h = h
        return self

    @classmethod
    def from_workload(cls, g):
        return cls(g.n, g.row_ptr, g.col, g.w)

    @classmethod
    def batch(cls, graphs):
        """lcd_graph_upload_batch: several independent graphs (workload
        Graph objects, all weighted or all unweighted) as one resident batch."""
        self = cls.__new__(cls)
        k = len(graphs)
        node_off = np.zeros(k + 1, np.int64)
        edge_off = np.zeros(k + 1, np.int64)
        for i, g in enumerate(graphs):
            node_off[i + 1] = node_off[i] + g.n
            edge_off[i + 1] = edge_off[i] + g.nnz
        rp = np.ascontiguousarray(np.concatenate([np.asarray(g.row_ptr, np.int32) for g in graphs]))
        cl = np.ascontiguousarray(np.concatenate([np.asarray(g.col, np.int32) for g in graphs]))
        weighted = [g.w is not None for g in graphs]
        if any(weighted) and not all(weighted):
            raise ValueError("a batch is either all weighted or all unweighted")
        w = (np.ascontiguousarray(np.concatenate([np.asarray(g.w, np.uint8) for g in graphs]))
             if all(weighted) else None)
        h = P()
        _check(library().lcd_graph_upload_batch(
            k, node_off.ctypes.data_as(P), edge_off.ctypes.data_as(P), rp.ctypes.data_as(P),
            cl.ctypes.data_as(P), None if w is None else w.ctypes.data_as(P), LCD_MEM_HOST, _stream(),
            ctypes.byref(h)), "lcd_graph_upload_batch")
        self._h = h
        self.n = int(node_off[-1])
        return self

    def batch_info(self) -> np.ndarray:
        """node_off of the member graphs ([0, n] for a plain graph)."""
        k = ctypes.c_int32()
        _check(library().lcd_graph_batch_info(self._h, ctypes.byref(k), None), "lcd_graph_batch_info")
        off = np.zeros(k.value + 1, np.int64)
        _check(library().lcd_graph_batch_info(self._h, ctypes.byref(k), off.ctypes.data_as(P)),
               "lcd_graph_batch_info")
        return off

    def info(self) -> dict:
        n = ctypes.c_int32()
        nnz = ctypes.c_int64()
        mk = ctypes.c_int64()
        vol = ctypes.c_int64()
        _check(library().lcd_graph_info(self._h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(mk),
                                        ctypes.byref(vol)), "lcd_graph_info")
        return dict(n=n.value, nnz=nnz.value, max_degree=mk.value, volume=vol.value)

    def untune(self):
        _check(library().lcd_graph_untune(self._h), "lcd_graph_untune")

    def free(self):
        if getattr(self, "_h", None):
            library().lcd_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Result:
    """The per-(seed set, scale) output of one sweep (lcd_result)."""

    def __init__(self, h, n: int):
        self._h = h
        self.n = n
        ns = ctypes.c_int32()
        S = ctypes.c_int32()
        _check(library().lcd_result_shape(h, ctypes.byref(ns), ctypes.byref(S)), "lcd_result_shape")
        self.n_sets = ns.value
        self.n_scales = S.value

    def sizes(self, s: int) -> int:
        t = ctypes.c_int64()
        _check(library().lcd_result_sizes(self._h, s, ctypes.byref(t)), "lcd_result_sizes")
        return t.value

    def membership(self, s: int):
        """(comm_ptr, members, k_in, vol, f) at scale s, device tensors."""
        tot = self.sizes(s)
        cp = torch.empty(self.n_sets + 1, dtype=torch.int32, device="cuda")
        m = torch.empty(max(tot, 1), dtype=torch.int32, device="cuda")
        k = torch.empty(max(self.n_sets, 1), dtype=torch.int64, device="cuda")
        v = torch.empty(max(self.n_sets, 1), dtype=torch.int64, device="cuda")
        f = torch.empty(max(self.n_sets, 1), dtype=torch.float64, device="cuda")
        _check(library().lcd_result_membership(self._h, s, _ptr(cp), _ptr(m), _ptr(k), _ptr(v), _ptr(f),
                                               LCD_MEM_DEVICE, _stream()), "lcd_result_membership")
        return cp, m[:tot], k[:self.n_sets], v[:self.n_sets], f[:self.n_sets]

    def delta(self, s: int):
        """(add_ptr, added, rem_ptr, removed) at scale s, device tensors: the
        ids that joined and left each set's community since scale s - 1
        (a sweep with output_mode=LCD_OUT_DELTA)."""
        na, nr = ctypes.c_int64(), ctypes.c_int64()
        _check(library().lcd_result_delta_sizes(self._h, s, ctypes.byref(na), ctypes.byref(nr)),
               "lcd_result_delta_sizes")
        ap = torch.empty(self.n_sets + 1, dtype=torch.int64, device="cuda")
        rp = torch.empty(self.n_sets + 1, dtype=torch.int64, device="cuda")
        a = torch.empty(max(na.value, 1), dtype=torch.int32, device="cuda")
        r = torch.empty(max(nr.value, 1), dtype=torch.int32, device="cuda")
        _check(library().lcd_result_delta(self._h, s, _ptr(ap), _ptr(a), _ptr(rp), _ptr(r), LCD_MEM_DEVICE,
                                          _stream()), "lcd_result_delta")
        return ap, a[:na.value], rp, r[:nr.value]

    def overlap(self, s: int):
        """(node_ptr, node_sets) at scale s, device tensors."""
        tot = self.sizes(s)
        npt = torch.empty(self.n + 1, dtype=torch.int32, device="cuda")
        nst = torch.empty(max(tot, 1), dtype=torch.int32, device="cuda")
        _check(library().lcd_result_overlap(self._h, s, _ptr(npt), _ptr(nst), LCD_MEM_DEVICE, _stream()),
               "lcd_result_overlap")
        return npt, nst[:tot]

    def nmi(self, s1: int, s2: int) -> float:
        """NMI of the community sets of scales s1 and s2 (lcd_result_nmi)."""
        out = ctypes.c_double()
        _check(library().lcd_result_nmi(self._h, s1, s2, ctypes.byref(out), _stream()), "lcd_result_nmi")
        return out.value

    def nmi_successive(self, p: int) -> np.ndarray:
        """NMI averaged over p successive scales (lcd_result_nmi_successive)."""
        out = np.zeros(max(self.n_scales - p + 1, 1), np.float64)
        _check(library().lcd_result_nmi_successive(self._h, p, out.ctypes.data_as(P), _stream()),
               "lcd_result_nmi_successive")
        return out[:self.n_scales - p + 1]

    def nmi_cover(self, s: int, cover) -> float:
        """NMI of scale s's community set with a cover (list of ascending
        node-id arrays), e.g. the planted communities."""
        ptr, mem = _cover_dev(cover)
        out = ctypes.c_double()
        _check(library().lcd_result_nmi_cover(self._h, s, int(ptr.numel()) - 1, _ptr(ptr), _ptr(mem),
                                              ctypes.byref(out), _stream()), "lcd_result_nmi_cover")
        return out.value

    def counters(self, per_record: bool = False):
        tot = (ctypes.c_uint64 * 4)()
        pr = None
        if per_record:
            pr = torch.empty(max(self.n_sets * self.n_scales * 4, 1), dtype=torch.int64, device="cuda")
        _check(library().lcd_result_counters(self._h, ctypes.cast(tot, P), _ptr(pr), LCD_MEM_DEVICE,
                                             _stream()), "lcd_result_counters")
        totals = [int(x) for x in tot]
        if per_record:
            return totals, pr[:self.n_sets * self.n_scales * 4].view(-1, 4)
        return totals

    def sets_to_numpy(self, set_ids) -> dict:
        """Every scale of the given seed sets, laid out like the oracle's
        run_sets() output for those sets (record q * S + s)."""
        ids = np.ascontiguousarray(set_ids, dtype=np.int32)
        S = self.n_scales
        R = ids.size * S
        off = np.zeros(max(R, 1), np.int64)
        cnt = np.zeros(max(R, 1), np.int32)
        K = np.zeros(max(R, 1), np.int64)
        V = np.zeros(max(R, 1), np.int64)
        f = np.zeros(max(R, 1), np.float64)
        ctr = np.zeros(max(R, 1) * 4, np.uint64)
        need = ctypes.c_int64()
        lib = library()
        _check(lib.lcd_result_sets(self._h, ids.ctypes.data_as(P), ids.size, off.ctypes.data_as(P),
                                   cnt.ctypes.data_as(P), None, 0, ctypes.byref(need), None, None,
                                   None, None), "lcd_result_sets")
        mem = np.zeros(max(need.value, 1), np.int32)
        _check(lib.lcd_result_sets(self._h, ids.ctypes.data_as(P), ids.size, off.ctypes.data_as(P),
                                   cnt.ctypes.data_as(P), mem.ctypes.data_as(P), mem.size,
                                   ctypes.byref(need), K.ctypes.data_as(P), V.ctypes.data_as(P),
                                   f.ctypes.data_as(P), ctr.ctypes.data_as(P)), "lcd_result_sets")
        return dict(members=mem[:need.value], off=off[:R], cnt=cnt[:R], K=K[:R], V=V[:R], f=f[:R],
                    ctr=ctr[:R * 4].reshape(R, 4), n_sets=ids.size, n_scales=S)

    def rerun(self):
        """lcd_result_rerun: the same sweep again into this result."""
        _check(library().lcd_result_rerun(self._h, _stream()), "lcd_result_rerun")
        return self

    def stats(self) -> dict:
        s = lcd_sweep_stats()
        _check(library().lcd_result_stats(self._h, ctypes.byref(s)), "lcd_result_stats")
        return s.as_dict()

    def free(self):
        if getattr(self, "_h", None):
            library().lcd_result_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def make_params(k_prune: int = 0, mode: int = LCD_PERSISTENT, lds_capacity: int = 0,
                waves_per_block: int = 0, blocks_per_cu: int = 0, use_graph: int = 0,
                pool_hint: int = 0, watchdog_ms: int = 0, spill_mode: int = 0,
                team_capacity: int = 0, team_waves: int = 0, grow_calls: int = 0,
                queue_min_entries: int = 0, output_mode: int = LCD_OUT_FULL) -> lcd_params:
    p = lcd_params()
    library().lcd_params_default(ctypes.byref(p))
    p.k_prune = k_prune
    p.mode = mode
    p.lds_capacity = lds_capacity
    p.waves_per_block = waves_per_block
    p.blocks_per_cu = blocks_per_cu
    p.use_graph = use_graph
    p.pool_hint = pool_hint
    if watchdog_ms:
        p.watchdog_ms = watchdog_ms
    p.spill_mode = spill_mode
    p.team_capacity = team_capacity
    p.team_waves = team_waves
    p.grow_calls = grow_calls
    p.queue_min_entries = queue_min_entries
    p.output_mode = output_mode
    return p


def lcd_sweep(graph: Graph, scales, seed_ptr, seed_nodes, params: Optional[lcd_params] = None,
              **kw) -> Result:
    """Grow every seed set through every scale (blocking).  Inputs may be
    numpy arrays or tensors; they are placed on the device first."""
    sc = _dev(scales, torch.float64)
    sp = _dev(seed_ptr, torch.int32)
    sn = _dev(seed_nodes, torch.int32)
    if sn.numel() == 0:
        sn = torch.zeros(1, dtype=torch.int32, device="cuda")
    prm = params if params is not None else make_params(**kw)
    h = P()
    _check(library().lcd_sweep(graph._h, _ptr(sc), int(sc.numel()), _ptr(sp), _ptr(sn),
                               int(sp.numel()) - 1, LCD_MEM_DEVICE, ctypes.byref(prm), _stream(),
                               ctypes.byref(h)), "lcd_sweep")
    return Result(h, graph.n)


def sweep_to_numpy(res: Result) -> dict:
    """Every record of a result as host arrays, laid out like the oracle's
    (record r = set * S + s; members of r at members[off[r]:off[r]+cnt[r]])."""
    S = res.n_scales
    ns = res.n_sets
    offs = np.zeros(ns * S, dtype=np.int64)
    cnt = np.zeros(ns * S, dtype=np.int32)
    K = np.zeros(ns * S, dtype=np.int64)
    V = np.zeros(ns * S, dtype=np.int64)
    f = np.zeros(ns * S, dtype=np.float64)
    chunks = []
    base = 0
    for s in range(S):
        cp, m, k, v, ff = res.membership(s)
        cp = cp.cpu().numpy().astype(np.int64)
        m = m.cpu().numpy()
        idx = np.arange(ns) * S + s
        offs[idx] = base + cp[:-1]
        cnt[idx] = np.diff(cp)
        K[idx] = k.cpu().numpy()
        V[idx] = v.cpu().numpy()
        f[idx] = ff.cpu().numpy()
        chunks.append(m)
        base += m.size
    members = np.concatenate(chunks) if chunks else np.zeros(0, np.int32)
    _, ctr = res.counters(per_record=True)
    return dict(members=members, off=offs, cnt=cnt, K=K, V=V, f=f,
                ctr=ctr.cpu().numpy().astype(np.uint64), n_sets=ns, n_scales=S)


def lcd_sweep_merge(graph: "Graph", scales, seed_ptr, seed_nodes, eta=(1, 2), params=None, **kw):
    """lcd_sweep_merge: the multi-scale loop with the check-and-merge phase."""
    lib = library()
    prm = params if params is not None else make_params(**kw)
    sc = np.ascontiguousarray(scales, dtype=np.float64)
    sp = np.ascontiguousarray(seed_ptr, dtype=np.int32)
    sn = np.ascontiguousarray(seed_nodes, dtype=np.int32)
    h = P()
    _check(lib.lcd_sweep_merge(graph._h, sc.ctypes.data_as(P), sc.size, sp.ctypes.data_as(P),
                               sn.ctypes.data_as(P), sp.size - 1, int(eta[0]), int(eta[1]), LCD_MEM_HOST,
                               ctypes.byref(prm), _stream(), ctypes.byref(h)), "lcd_sweep_merge")
    return Result(h, graph.n)


def merged_into(res: "Result") -> np.ndarray:
    """into[R] in record order (set * S + s): -1 live, else the live id."""
    S, ns = res.n_scales, res.n_sets
    out = np.zeros((ns, S), np.int32)
    col = np.zeros(max(ns, 1), np.int32)
    for s in range(S):
        _check(library().lcd_result_merged_into(res._h, s, col.ctypes.data_as(P)), "lcd_result_merged_into")
        out[:, s] = col[:ns]
    return out.reshape(-1)


def lcd_seeds(graph: "Graph", perm, rule: int = 1) -> np.ndarray:
    """Seed selection (rule 1 or 2) on the device, visiting nodes in the order
    perm; the seeds in order of selection (host array)."""
    p = np.ascontiguousarray(perm, dtype=np.int32)
    out = np.zeros(max(p.size, 1), np.int32)
    k = ctypes.c_int32()
    _check(library().lcd_seeds(graph._h, int(rule), p.ctypes.data_as(P), LCD_MEM_HOST, _stream(),
                               out.ctypes.data_as(P), ctypes.byref(k)), "lcd_seeds")
    return out[:k.value].copy()


def _cover_dev(cover):
    sizes = [len(c) for c in cover]
    ptr = np.zeros(len(cover) + 1, np.int32)
    np.cumsum(sizes, out=ptr[1:])
    mem = (np.concatenate([np.asarray(c, np.int32) for c in cover]) if ptr[-1] > 0
           else np.zeros(1, np.int32))
    return _dev(ptr, torch.int32), _dev(mem, torch.int32)


def lcd_cover_nmi(n: int, cover_x, cover_y) -> float:
    """NMI of two covers of n nodes on the device (lcd_cover_nmi); each cover
    a list of strictly ascending node-id arrays."""
    px, mx = _cover_dev(cover_x)
    py, my = _cover_dev(cover_y)
    out = ctypes.c_double()
    _check(library().lcd_cover_nmi(int(n), int(px.numel()) - 1, _ptr(px), _ptr(mx), int(py.numel()) - 1,
                                   _ptr(py), _ptr(my), ctypes.byref(out), _stream()), "lcd_cover_nmi")
    return out.value


def lcd_sweep_into(graph: "Graph", scales, seed_ptr, seed_nodes, members_cap: int, out: Optional[dict] = None,
                   params: Optional[lcd_params] = None, **kw) -> dict:
    """lcd_sweep_into: the sweep with caller-owned device outputs and no
    allocation inside the library.  ``out`` may hold the output tensors
    (rec_off, rec_cnt, rec_k, rec_v, rec_f, rec_ctr, members) from an earlier
    call of at least this size; missing ones are allocated here, by the
    caller's side.  Returns the tensors and ``members_used``."""
    sc = _dev(scales, torch.float64)
    sp = _dev(seed_ptr, torch.int32)
    sn = _dev(seed_nodes, torch.int32)
    ns = int(sp.numel()) - 1
    S = int(sc.numel())
    R = max(ns * S, 1)
    o = dict(out or {})
    spec = dict(rec_off=(R, torch.int64), rec_cnt=(R, torch.int32), rec_k=(R, torch.int64),
                rec_v=(R, torch.int64), rec_f=(R, torch.float64), rec_ctr=(4 * R, torch.int64),
                members=(max(int(members_cap), 1), torch.int32))
    for k, (size, dt) in spec.items():
        if k not in o or o[k].numel() < size:
            o[k] = torch.empty(size, dtype=dt, device="cuda")
    if sn.numel() == 0:
        sn = torch.zeros(1, dtype=torch.int32, device="cuda")
    prm = params if params is not None else make_params(**kw)
    used = ctypes.c_int64()
    _check(library().lcd_sweep_into(graph._h, _ptr(sc), S, _ptr(sp), _ptr(sn), ns,
                                    int(seed_ptr[-1]) if ns > 0 else 0, ctypes.byref(prm),
                                    _ptr(o["rec_off"]), _ptr(o["rec_cnt"]), _ptr(o["rec_k"]), _ptr(o["rec_v"]),
                                    _ptr(o["rec_f"]), _ptr(o["rec_ctr"]), _ptr(o["members"]), int(members_cap),
                                    ctypes.byref(used), _stream()), "lcd_sweep_into")
    o["members_used"] = used.value
    return o


def lcd_sweep_batch(graph: "Graph", scales, seed_ptr, seed_nodes, seed_graph, params=None, **kw):
    """lcd_sweep_batch: seeds local to member graph seed_graph[j]; member
    lists of the result are in batch ids (node_off[graph] + local id)."""
    lib = library()
    prm = params if params is not None else make_params(**kw)
    sc = np.ascontiguousarray(scales, dtype=np.float64)
    sp = np.ascontiguousarray(seed_ptr, dtype=np.int32)
    sn = np.ascontiguousarray(seed_nodes, dtype=np.int32)
    sg = np.ascontiguousarray(seed_graph, dtype=np.int32)
    h = P()
    _check(lib.lcd_sweep_batch(graph._h, sc.ctypes.data_as(P), sc.size, sp.ctypes.data_as(P),
                               sn.ctypes.data_as(P), sg.ctypes.data_as(P), sp.size - 1, LCD_MEM_HOST,
                               ctypes.byref(prm), _stream(), ctypes.byref(h)), "lcd_sweep_batch")
    return Result(h, graph.n)


def lcd_tune(graph: "Graph", scales, seed_ptr, seed_nodes, **base) -> dict:
    """Autotune the launch sizing for this graph and seed sets (the graph
    keeps the choice for later sweeps with default params)."""
    lib = library()
    sc = np.ascontiguousarray(scales, dtype=np.float64)
    sp = np.ascontiguousarray(seed_ptr, dtype=np.int32)
    sn = np.ascontiguousarray(seed_nodes, dtype=np.int32)
    prm = make_params(**base)
    rep = lcd_tune_report()
    _check(lib.lcd_tune(graph._h, sc.ctypes.data_as(P), sc.size, sp.ctypes.data_as(P),
                        sn.ctypes.data_as(P), sp.size - 1, LCD_MEM_HOST, ctypes.byref(prm), _stream(),
                        ctypes.byref(rep)), "lcd_tune")
    keys = ("lds_capacity", "spill_mode", "team_capacity", "team_waves")
    return dict(best={k: getattr(rep.best, k) for k in keys}, ms_best=rep.ms_best,
                sample_stride=rep.sample_stride, full_checked=bool(rep.full_checked),
                tried=[dict({k: getattr(rep.tried[i], k) for k in keys}, ms=round(rep.ms[i], 3))
                       for i in range(rep.n_tried)])


# ---------------------------------------------------------------------------
# Query server
# ---------------------------------------------------------------------------

class Server:
    """lcd_server_*: (seed set, alpha) queries answered by a resident graph,
    batched as they arrive by the library's worker thread."""

    def __init__(self, graph: "Graph", mem_budget: int = 0, max_slots: int = 0, **kw):
        lib = library()
        prm = make_params(**kw) if kw else None
        h = P()
        _check(lib.lcd_server_create(graph._h, int(mem_budget), int(max_slots),
                                     ctypes.byref(prm) if prm is not None else None,
                                     ctypes.byref(h)), "lcd_server_create")
        self._h = h
        self.graph = graph

    def submit(self, seeds, alpha: float) -> int:
        a = np.ascontiguousarray(seeds, dtype=np.int32)
        t = ctypes.c_uint64()
        _check(library().lcd_server_submit(self._h, a.ctypes.data_as(P), a.size, float(alpha),
                                           ctypes.byref(t)), "lcd_server_submit")
        return t.value

    def poll(self, ticket: int):
        """None while the query runs, else a dict with members and info."""
        lib = library()
        info = lcd_query_info()
        s = lib.lcd_server_poll(self._h, ticket, None, 0, ctypes.byref(info))
        if s == LCD_EAGAIN:
            return None
        if s == LCD_ECAPACITY or (s == LCD_OK and info.n_members > 0):
            mem = np.zeros(max(info.n_members, 1), np.int32)
            s = lib.lcd_server_poll(self._h, ticket, mem.ctypes.data_as(P), mem.size,
                                    ctypes.byref(info))
            _check(s, "lcd_server_poll")
            mem = mem[:info.n_members]
        else:
            _check(s, "lcd_server_poll")
            mem = np.zeros(0, np.int32)
        return dict(members=mem, K=info.k_in, V=info.vol, f=info.f,
                    ctr=np.array(list(info.ctr), dtype=np.uint64),
                    t_submit_ns=info.t_submit_ns, t_start_ns=info.t_start_ns,
                    t_done_ns=info.t_done_ns, batch_size=info.batch_size, lane=info.lane)

    def wait(self, ticket: int, timeout_ms: int = -1) -> bool:
        s = library().lcd_server_wait(self._h, ticket, int(timeout_ms))
        if s == LCD_EAGAIN:
            return False
        _check(s, "lcd_server_wait")
        return True

    def cancel(self, ticket: int) -> bool:
        """Withdraw a query: True if it was withdrawn (its ticket ends with
        LCD_ECANCELED), False if it had already completed."""
        s = library().lcd_server_cancel(self._h, ticket)
        if s == LCD_ESTATE:
            return False
        _check(s, "lcd_server_cancel")
        return True

    def result(self, ticket: int, timeout_ms: int = -1):
        if not self.wait(ticket, timeout_ms):
            raise TimeoutError("query %d not done after %d ms" % (ticket, timeout_ms))
        return self.poll(ticket)

    def stats(self) -> dict:
        st = lcd_server_stats()
        _check(library().lcd_server_get_stats(self._h, ctypes.byref(st)), "lcd_server_get_stats")
        return st.as_dict()

    def close(self):
        if self._h:
            _check(library().lcd_server_destroy(self._h), "lcd_server_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
