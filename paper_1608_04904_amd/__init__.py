"""MI355X (gfx950) solvent hot path of hybrid Reactive MPCD + MD.

Thin binding over the C ABI of ``librmpmd.so`` (include/rmpmd.h) with the
same names: ``init_system``, ``step``, ``observables``, ``get_state``,
``set_state``, ``workspace_bytes`` and the batch calls.  PyTorch provides the
device memory (a uint8 workspace tensor) and the stream; all arithmetic of
the method runs in the library's HIP kernels.  There is no CPU fallback: on a
machine without the library or a GPU these calls raise.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi
from ._capi import RmpError, check, make_params, obs_dict

__all__ = ["System", "Batch", "workspace_bytes", "analysis_bytes", "init_system", "RmpError"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("rmpmd needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def workspace_bytes(params: dict) -> int:
    q = make_params(params)
    st = C.c_int32(0)
    n = _capi.lib().rmp_workspace_bytes(C.byref(q), C.byref(st))
    check(st.value, "rmp_workspace_bytes")
    return int(n)


def _alloc(nbytes: int, device):
    torch = _torch()
    # 256-byte alignment is guaranteed by the caching allocator
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def analysis_bytes(params: dict, analysis: dict) -> int:
    q, a = make_params(params), _capi.make_analysis_params(analysis)
    st = C.c_int32(0)
    n = _capi.lib().rmp_analysis_bytes(C.byref(q), C.byref(a), C.byref(st))
    check(st.value, "rmp_analysis_bytes")
    return int(n)


class _Analysis:
    """Host side of one attached dimer analysis: its device buffer and the
    host arrays it is read into."""

    def __init__(self, params: dict, analysis: dict, device):
        self.a = _capi.make_analysis_params(analysis)
        self.nb = len(params["bonds"])
        self.buf = _alloc(analysis_bytes(params, analysis), device)
        cap, nz, nr = self.a.series_cap, self.a.hist_nz, self.a.hist_nr
        self.md_step = np.zeros(cap, dtype=np.int64)
        self.series = np.zeros((cap, self.nb, _capi.SERIES_FIELDS))
        self.hist = np.zeros((self.nb, 2, nz, nr), dtype=np.uint64)

    def out(self) -> _capi.AnalysisOut:
        o = _capi.AnalysisOut()
        o.md_step, o.series, o.hist = _ptr(self.md_step), _ptr(self.series), _ptr(self.hist)
        return o

    def result(self, o: _capi.AnalysisOut) -> dict:
        k = int(o.n_samples)
        return dict(n_samples=k, n_dropped=int(o.n_dropped), md_step=self.md_step[:k].copy(),
                    series=self.series[:k].copy(), hist=self.hist.copy())


class _StateBuffers:
    def __init__(self, n: int, nc: int):
        self.x = np.zeros((3, n))
        self.v = np.zeros((3, n))
        self.id = np.zeros(n, dtype=np.uint32)
        self.state = np.zeros(n, dtype=np.uint8)
        self.X = np.zeros((max(nc, 1), 3))
        self.V = np.zeros((max(nc, 1), 3))
        self.nc = nc

    def host_state(self, md=0, coll=0) -> _capi.HostState:
        h = _capi.HostState()
        h.x, h.v = _ptr(self.x), _ptr(self.v)
        h.id, h.state = _ptr(self.id), _ptr(self.state)
        h.X, h.V = _ptr(self.X), _ptr(self.V)
        h.md_step, h.coll_step = int(md), int(coll)
        return h

    def to_dict(self, h) -> dict:
        return dict(x=self.x.copy(), v=self.v.copy(), id=self.id.copy(),
                    state=self.state.copy(), X=self.X[: self.nc].copy(),
                    V=self.V[: self.nc].copy(), md_step=h.md_step, coll_step=h.coll_step)


def _fill(buf: _StateBuffers, s: dict):
    n = buf.id.size
    buf.x[:] = np.asarray(s["x"], dtype=np.float64).reshape(3, n)
    buf.v[:] = np.asarray(s["v"], dtype=np.float64).reshape(3, n)
    buf.id[:] = np.asarray(s["id"], dtype=np.uint32)
    buf.state[:] = np.asarray(s["state"], dtype=np.uint8)
    if buf.nc:
        buf.X[: buf.nc] = np.asarray(s["X"], dtype=np.float64).reshape(buf.nc, 3)
        buf.V[: buf.nc] = np.asarray(s["V"], dtype=np.float64).reshape(buf.nc, 3)


def check_state(params: dict, s: dict) -> int:
    """rmp_check_state: the library's host-side check of a state for these
    parameters (no device needed); returns the status (0 = acceptable)."""
    n, nc = int(params["n_solvent"]), len(params["colloids"])
    b = _StateBuffers(n, nc)
    _fill(b, s)
    h = b.host_state(s.get("md_step", 0), s.get("coll_step", 0))
    q = _capi.make_params(params)
    return int(_capi.lib().rmp_check_state(C.byref(q), C.byref(h)))


class System:
    """One simulated system (``rmp_init_system`` ... ``rmp_destroy``)."""

    def __init__(self, params: dict, seed: int, device="cuda:0", stream=None):
        torch = _torch()
        self.params = params
        self.seed = int(seed)
        self.device = torch.device(device)
        self.n = int(params["n_solvent"])
        self.nc = len(params["colloids"])
        self._q = make_params(params)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ws = _alloc(workspace_bytes(params), self.device)
        h = C.c_void_p()
        check(_capi.lib().rmp_init_system(
            C.byref(self._q), self.seed, C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
            C.c_void_p(self.stream.cuda_stream), C.byref(h)), "rmp_init_system")
        self.h = h
        self._buf = None
        self._an = None

    def close(self):
        if getattr(self, "h", None):
            _capi.lib().rmp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n_md: int, n_collide: int = 1):
        check(_capi.lib().rmp_step(self.h, int(n_md), int(n_collide)), "rmp_step")

    def observables(self, raise_on_flags: bool = True) -> dict:
        o = _capi.Obs()
        st = _capi.lib().rmp_observables(self.h, C.byref(o))
        if st not in (_capi.OK, _capi.EDEVICE) or (st == _capi.EDEVICE and raise_on_flags):
            raise RmpError(st, "rmp_observables", o.flags)
        return obs_dict(o, self.nc)

    def observables_noalloc(self, raise_on_flags: bool = True) -> dict:
        """rmp_observables_noalloc: the same results from the library's
        static device scratch (no allocation in the call)."""
        o = _capi.Obs()
        st = _capi.lib().rmp_observables_noalloc(self.h, C.byref(o))
        if st not in (_capi.OK, _capi.EDEVICE) or (st == _capi.EDEVICE and raise_on_flags):
            raise RmpError(st, "rmp_observables_noalloc", o.flags,
                           detail=st in (_capi.ENOMEM, _capi.ESTATE))
        return obs_dict(o, self.nc)

    def _buffers(self):
        if self._buf is None:
            self._buf = _StateBuffers(self.n, self.nc)
        return self._buf

    def get_state(self) -> dict:
        b = self._buffers()
        h = b.host_state()
        check(_capi.lib().rmp_get_state(self.h, C.byref(h)), "rmp_get_state")
        return b.to_dict(h)

    def set_state(self, s: dict):
        b = self._buffers()
        _fill(b, s)
        h = b.host_state(s.get("md_step", 0), s.get("coll_step", 0))
        check(_capi.lib().rmp_set_state(self.h, C.byref(h)), "rmp_set_state")

    def set_tuning(self, **kw):
        t = _capi.Tuning(*([-1] * len(_capi.Tuning._fields_)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        check(_capi.lib().rmp_set_tuning(self.h, C.byref(t)), "rmp_set_tuning")

    # dimer analysis (rmp_analysis_*)
    def analysis_attach(self, **analysis):
        an = _Analysis(self.params, analysis, self.device)
        check(_capi.lib().rmp_analysis_attach(self.h, C.byref(an.a), C.c_void_p(an.buf.data_ptr()),
                                              an.buf.numel()), "rmp_analysis_attach")
        self._an = an

    def analysis_detach(self):
        check(_capi.lib().rmp_analysis_detach(self.h), "rmp_analysis_detach")
        self._an = None

    def analysis_read(self) -> dict:
        # nothing attached: the library reports it (null outputs are not written)
        o = self._an.out() if self._an else _capi.AnalysisOut()
        check(_capi.lib().rmp_analysis_read(self.h, C.byref(o)), "rmp_analysis_read")
        return self._an.result(o)

    def analysis_msd(self, max_lag: int) -> np.ndarray:
        nb = self._an.nb if self._an else len(self.params["bonds"])
        m = np.zeros((max(nb, 1), int(max_lag) + 1))
        check(_capi.lib().rmp_analysis_msd(self.h, int(max_lag), _ptr(m)), "rmp_analysis_msd")
        return m

    def get_tuning(self) -> dict:
        t = _capi.Tuning()
        check(_capi.lib().rmp_get_tuning(self.h, C.byref(t)), "rmp_get_tuning")
        return {k: getattr(t, k) for k, _ in _capi.Tuning._fields_}

    def profile(self, enable: bool):
        check(_capi.lib().rmp_profile(self.h, int(bool(enable))), "rmp_profile")

    def profile_read(self) -> dict:
        cap = 16
        names = (C.c_char_p * cap)()
        ms = (C.c_double * cap)()
        cnt = (C.c_int64 * cap)()
        m = _capi.lib().rmp_profile_read(self.h, names, ms, cnt, cap)
        return {names[i].decode(): (ms[i], cnt[i]) for i in range(m)}


def init_system(params: dict, seed: int, device="cuda:0", stream=None) -> System:
    return System(params, seed, device=device, stream=stream)


class Batch:
    """Replicas advanced together (``rmp_batch_*``); slots are filled and
    emptied between ticks.  Each replica owns a workspace tensor."""

    def __init__(self, n_slots: int, precision: int = 64, device="cuda:0", stream=None):
        torch = _torch()
        self.device = torch.device(device)
        self.n_slots = int(n_slots)
        self.precision = int(precision)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctl = _alloc(_capi.lib().rmp_batch_ctl_bytes(self.n_slots), self.device)
        h = C.c_void_p()
        check(_capi.lib().rmp_batch_create(
            self.n_slots, self.precision, C.c_void_p(self.ctl.data_ptr()), self.ctl.numel(),
            C.c_void_p(self.stream.cuda_stream), C.byref(h)), "rmp_batch_create")
        self.h = h
        self.slots = [None] * self.n_slots

    def close(self):
        if getattr(self, "h", None):
            _capi.lib().rmp_batch_destroy(self.h)
            self.h = None
            self.slots = [None] * self.n_slots

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_slot(self, slot: int, params: dict, seed: int, n_md: int, workspace=None):
        q = make_params(params)
        need = workspace_bytes(params)
        ws = workspace if workspace is not None else _alloc(need, self.device)
        check(_capi.lib().rmp_batch_set_slot(self.h, int(slot), C.byref(q), int(seed), int(n_md),
                                             C.c_void_p(ws.data_ptr()), ws.numel()),
              "rmp_batch_set_slot")
        self.slots[slot] = dict(params=params, ws=ws, q=q, buf=None, an=None,
                                n=int(params["n_solvent"]), nc=len(params["colloids"]))

    def clear_slot(self, slot: int):
        check(_capi.lib().rmp_batch_clear_slot(self.h, int(slot)), "rmp_batch_clear_slot")
        self.slots[slot] = None

    def step(self, n_ticks: int = 1):
        check(_capi.lib().rmp_batch_step(self.h, int(n_ticks)), "rmp_batch_step")

    def observables(self, slot: int, raise_on_flags: bool = True) -> dict:
        o = _capi.Obs()
        st = _capi.lib().rmp_batch_slot_observables(self.h, int(slot), C.byref(o))
        if st not in (_capi.OK, _capi.EDEVICE) or (st == _capi.EDEVICE and raise_on_flags):
            raise RmpError(st, "rmp_batch_slot_observables", o.flags)
        return obs_dict(o, self.slots[slot]["nc"])

    def _buffers(self, slot):
        s = self.slots[slot]
        if s["buf"] is None:
            s["buf"] = _StateBuffers(s["n"], s["nc"])
        return s["buf"]

    def get_state(self, slot: int) -> dict:
        b = self._buffers(slot)
        h = b.host_state()
        check(_capi.lib().rmp_batch_get_state(self.h, int(slot), C.byref(h)), "rmp_batch_get_state")
        return b.to_dict(h)

    def set_state(self, slot: int, s: dict):
        b = self._buffers(slot)
        _fill(b, s)
        h = b.host_state(s.get("md_step", 0), s.get("coll_step", 0))
        check(_capi.lib().rmp_batch_set_state(self.h, int(slot), C.byref(h)), "rmp_batch_set_state")

    def set_tuning(self, **kw):
        t = _capi.Tuning(*([-1] * len(_capi.Tuning._fields_)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        check(_capi.lib().rmp_batch_set_tuning(self.h, C.byref(t)), "rmp_batch_set_tuning")

    def set_slot_tuning(self, slot: int, collide_cells: int):
        t = _capi.Tuning(-1, -1, int(collide_cells), *([-1] * (len(_capi.Tuning._fields_) - 3)))
        check(_capi.lib().rmp_batch_set_slot_tuning(self.h, int(slot), C.byref(t)),
              "rmp_batch_set_slot_tuning")

    # dimer analysis of one slot (rmp_batch_analysis_*)
    def analysis_attach(self, slot: int, **analysis):
        an = _Analysis(self.slots[slot]["params"], analysis, self.device)
        check(_capi.lib().rmp_batch_analysis_attach(self.h, int(slot), C.byref(an.a),
                                                    C.c_void_p(an.buf.data_ptr()), an.buf.numel()),
              "rmp_batch_analysis_attach")
        self.slots[slot]["an"] = an

    def analysis_detach(self, slot: int):
        check(_capi.lib().rmp_batch_analysis_detach(self.h, int(slot)), "rmp_batch_analysis_detach")
        self.slots[slot]["an"] = None

    def analysis_read(self, slot: int) -> dict:
        an = self.slots[slot]["an"]
        o = an.out() if an else _capi.AnalysisOut()
        check(_capi.lib().rmp_batch_analysis_read(self.h, int(slot), C.byref(o)),
              "rmp_batch_analysis_read")
        return an.result(o)

    def analysis_msd(self, slot: int, max_lag: int) -> np.ndarray:
        an = self.slots[slot]["an"]
        nb = an.nb if an else len(self.slots[slot]["params"]["bonds"])
        m = np.zeros((max(nb, 1), int(max_lag) + 1))
        check(_capi.lib().rmp_batch_analysis_msd(self.h, int(slot), int(max_lag), _ptr(m)),
              "rmp_batch_analysis_msd")
        return m

