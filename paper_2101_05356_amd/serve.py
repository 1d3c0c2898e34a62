"""Python handle of the reconstruction server (fr_server_* of include/fr.h).

The scheduling (admission by slot and HBM budget, batched steps, retirement,
failure detection, latency statistics) runs in the library's worker thread;
this module only marshals arguments.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import FrRequest, FrResult, FrServerOpts, FrStats, check, lib
from .recon import JobSpec, Model

STATE_NAMES = {_lib.FR_REQ_QUEUED: "queued", _lib.FR_REQ_RUNNING: "running", _lib.FR_REQ_DONE: "done",
               _lib.FR_REQ_FAILED: "failed", _lib.FR_REQ_CANCELLED: "cancelled"}


def _host(a, dtype=np.float32):
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=dtype)


class Server:
    # Work cap measured on the face workload mix (128^2..512^2, 4..32 spp, 72
    # lights): past ~8e8 nominal rays per step, stepping more requests
    # together raises the completion rate little and delays every request.
    DEFAULT_WORK_CAP = 8.0e8

    def __init__(self, model: Model, hbm_budget: int, max_slots: int = 32, quantum: int = 10, use_graph=True,
                 work_cap: float = DEFAULT_WORK_CAP):
        """work_cap: nominal rays per step (W*H*spp*(1+lights) summed over the
        requests stepped together) admitted at most; 0 = no cap."""
        self.model = model
        o = FrServerOpts()
        o.hbm_budget, o.max_slots, o.quantum, o.use_graph = int(hbm_budget), int(max_slots), int(quantum), \
            int(bool(use_graph))
        o.work_cap = float(work_cap)
        h = ctypes.c_void_p()
        check(lib().fr_server_create(model.h, ctypes.byref(o), ctypes.byref(h)), model.ctx.h, "fr_server_create")
        self.h = h
        self.jobs = {}

    def submit(self, job: JobSpec, n_steps: int) -> int:
        """Queue a reconstruction of `n_steps` Adam steps; inputs are copied.
        Pass host arrays: a device tensor is first copied to the host, and
        that copy waits for work already queued on the device."""
        lt, cam = job.lights, job.camera
        arrays = dict(cam=_host(np.concatenate([np.asarray(cam.R, np.float32).reshape(9),
                                                np.asarray(cam.T, np.float32)])),
                      p0=_host(lt.p0), e1=_host(lt.e1), e2=_host(lt.e2), shape=_host(lt.shape, np.int32),
                      target=_host(job.target), params=_host(job.params), lr=_host(job.lr))
        r = FrRequest()
        d = r.job
        d.width, d.height, d.spp, d.n_lights = job.W, job.H, job.spp, job.L
        d.edge_samples, d.smooth, d.brdf_variant, d.hist_cap = job.edge_samples, int(job.smooth), \
            job.brdf_variant, max(job.hist_cap, n_steps)
        d.seed, d.fov_y = job.seed, float(cam.fov_y)
        d.shadow_edge_samples = job.shadow_edge_samples
        ptr = lambda k: arrays[k].ctypes.data_as(ctypes.c_void_p).value
        d.cam, d.light_p0, d.light_e1, d.light_e2 = ptr("cam"), ptr("p0"), ptr("e1"), ptr("e2")
        d.light_shape, d.target, d.params, d.lr = ptr("shape"), ptr("target"), ptr("params"), ptr("lr")
        r.n_steps = int(n_steps)
        rid = ctypes.c_uint64()
        check(lib().fr_server_submit(self.h, ctypes.byref(r), ctypes.byref(rid)), self.model.ctx.h,
              "fr_server_submit")
        self.jobs[rid.value] = (job, int(n_steps))
        return rid.value

    def poll(self, rid: int, want_params=True) -> dict:
        job, n_steps = self.jobs[rid]
        res = FrResult()
        params = np.zeros(self.model.n_param(job.L), np.float32) if want_params else None
        losses = np.zeros(n_steps, np.float32)
        c = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        check(lib().fr_server_poll(self.h, rid, ctypes.byref(res), c(params), c(losses)), self.model.ctx.h,
              "fr_server_poll")
        out = {f: getattr(res, f) for f, _ in FrResult._fields_}
        out["state_name"] = STATE_NAMES.get(res.state, "?")
        if res.state in (_lib.FR_REQ_DONE, _lib.FR_REQ_FAILED) and res.n_losses > 0:
            out["params"] = params
            out["losses"] = losses[:res.n_losses]
        return out

    def cancel(self, rid: int):
        check(lib().fr_server_cancel(self.h, rid), self.model.ctx.h, "fr_server_cancel")

    def forget(self, rid: int):
        check(lib().fr_server_forget(self.h, rid), self.model.ctx.h, "fr_server_forget")
        del self.jobs[rid]

    def wait(self, timeout_s: float = 600.0) -> bool:
        return lib().fr_server_wait(self.h, float(timeout_s)) == _lib.FR_OK

    def clock(self) -> float:
        return float(lib().fr_server_clock(self.h))

    def stats(self) -> dict:
        s = FrStats()
        check(lib().fr_server_stats(self.h, ctypes.byref(s)), self.model.ctx.h, "fr_server_stats")
        return {f: getattr(s, f) for f, _ in FrStats._fields_ if f != "pad_"}

    def close(self):
        if getattr(self, "h", None) and _lib is not None and _lib._lib is not None:
            _lib._lib.fr_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()
