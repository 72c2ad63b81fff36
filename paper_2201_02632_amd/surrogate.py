"""Profile-table surrogate (an addition to the paper's method): training,
inference and exact fallback, driving the library's kernels.

All arithmetic runs in libbp.so (bp_mlp_*, bp_surrogate_*): this module holds
device buffers (torch tensors), draws the training batches' indices, and
sequences the calls.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import (MLP_IN, MLP_OUT, S_OUT_OF_DOMAIN, SOL_NFIELDS, META_NFIELDS, MLP_NQ, SUR_ARRAYS, SUR_TABLES, _check,
               _comp_ptrs, _lib, _ptr, _stream, _with_workspace, _ws_for, Workspace, default_params, icm_solve,
               profile_tables, surrogate_solve)


def _f64(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


class Surrogate:
    """MLP (3 -> 256 -> 256 -> 256 -> 144) with FP32 master weights, a BF16 compute copy and Adam state, all
    in one device state buffer that the library lays out (bp_surrogate_state_bytes); the attributes w, wb,
    m, v, g, mean and std are views into it."""

    def __init__(self, params=None, device="cuda", seed=0):
        self.params = params or default_params()
        self.dev = torch.device(device)
        self.np = int(_lib.bp_mlp_nparams())
        self.state = torch.empty(int(_lib.bp_surrogate_state_bytes()), dtype=torch.uint8, device=self.dev)
        off = {a: int(_lib.bp_surrogate_state_offset(k)) for k, a in enumerate(SUR_ARRAYS)}

        def view(a, n, dt, size):
            return self.state[off[a]:off[a] + n * size].view(dt)
        self.w = view("W", self.np, torch.float32, 4)
        self.wb = view("WBF16", self.np, torch.int16, 2)
        self.m = view("M", self.np, torch.float32, 4)
        self.v = view("V", self.np, torch.float32, 4)
        self.g = view("G", self.np, torch.float32, 4)
        self.mean = view("MEAN", MLP_OUT, torch.float32, 4)
        self.std = view("STD", MLP_OUT, torch.float32, 4)
        self.step = 0
        _check(_lib.bp_surrogate_init(_ptr(self.state), int(seed) & 0xFFFFFFFFFFFFFFFF, _stream()),
               "bp_surrogate_init")

    # -- parameters -------------------------------------------------------
    def _layout(self):
        H, I, O = 256, MLP_IN, MLP_OUT
        sizes = [("W1", H * I), ("b1", H), ("W2", H * H), ("b2", H), ("W3", H * H), ("b3", H), ("W4", O * H),
                 ("b4", O)]
        off, out = 0, {}
        for name, n in sizes:
            out[name] = (off, n)
            off += n
        assert off == self.np
        return out

    def to_blob(self) -> bytes:
        """The surrogate as a flat host blob (bp_surrogate_save)."""
        blob = (C.c_uint8 * int(_lib.bp_surrogate_blob_bytes()))()
        _check(_lib.bp_surrogate_save(_ptr(self.state), self.step, blob, len(blob), _stream()), "bp_surrogate_save")
        return bytes(blob)

    def from_blob(self, data: bytes):
        buf = (C.c_uint8 * len(data)).from_buffer_copy(data)
        step = C.c_int64(0)
        _check(_lib.bp_surrogate_load(_ptr(self.state), buf, len(buf), C.byref(step), _stream()), "bp_surrogate_load")
        self.step = step.value

    def save(self, path):
        with open(path, "wb") as f:
            f.write(self.to_blob())

    def load(self, path):
        with open(path, "rb") as f:
            self.from_blob(f.read())

    # -- kernels ------------------------------------------------------------
    def features(self, M, c, z):
        n = M.numel()
        x = torch.empty((n, MLP_IN), dtype=torch.float32, device=self.dev)
        _check(_lib.bp_surrogate_features(n, _ptr(M), _ptr(c), _ptr(z), _ptr(x), _stream()), "features")
        return x

    def forward(self, x, act=None):
        n = x.shape[0]
        y = torch.empty((n, MLP_OUT), dtype=torch.float32, device=self.dev)
        if act is None:
            act = torch.empty(int(_lib.bp_mlp_act_bytes(n)), dtype=torch.uint8, device=self.dev)
        _check(_lib.bp_mlp_forward(_ptr(self.w), _ptr(self.wb), n, _ptr(x), _ptr(y), _ptr(act), _stream()),
               "bp_mlp_forward")
        return y, act

    def predict(self, x):
        """Network outputs for many rows: the fused inference kernel (no activations stored)."""
        n = x.shape[0]
        y = torch.empty((n, MLP_OUT), dtype=torch.float32, device=self.dev)
        _check(_lib.bp_mlp_infer(_ptr(self.w), _ptr(self.wb), n, _ptr(x), _ptr(y), _stream()), "bp_mlp_infer")
        return y

    def backward(self, x, act, dy, ws=None):
        n = x.shape[0]
        need = int(_lib.bp_mlp_backward_ws_bytes(n))
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=self.dev)
        _check(_lib.bp_mlp_backward(_ptr(self.w), _ptr(self.wb), n, _ptr(x), _ptr(act), _ptr(dy), _ptr(self.g),
                                    _ptr(ws), ws.numel(), _stream()), "bp_mlp_backward")
        return self.g, ws

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        _check(_lib.bp_mlp_adam(self.np, _ptr(self.w), _ptr(self.m), _ptr(self.v), _ptr(self.g), _ptr(self.wb),
                                float(lr), b1, b2, eps, self.step, _stream()), "bp_mlp_adam")

    # -- training set from the exact path -------------------------------------
    def training_set(self, M, c, z):
        """Exact solve + tables -> (features, targets) on the device; rows of failed solves are NaN."""
        M, c, z = (_f64(a, self.dev) for a in (M, c, z))
        sol, st = icm_solve(self.params, M, c, z)
        tab, meta = profile_tables(self.params, sol, st)
        n = M.numel()
        t = torch.empty((n, MLP_OUT), dtype=torch.float32, device=self.dev)
        _check(_lib.bp_surrogate_targets(C.byref(self.params), n, _ptr(sol), _ptr(st), _ptr(tab), _ptr(meta), _ptr(t),
                                         _stream()), "targets")
        return self.features(M, c, z), t

    def set_stats(self, t):
        _check(_lib.bp_surrogate_stats(t.shape[0], _ptr(t), _ptr(self.mean), _ptr(self.std), _stream()), "stats")

    def fit(self, x, t, steps, batch=4096, lr=2e-3, lr_end=2e-5, seed=0, log_every=0):
        """Adam on the weighted MSE of standardised targets with a cosine learning-rate decay,
        run as a device-side loop (one library call per logging interval)."""
        n = x.shape[0]
        need = int(_lib.bp_surrogate_train_ws_bytes(batch))
        ws = torch.empty(need, dtype=torch.uint8, device=self.dev)
        loss = torch.empty(batch, dtype=torch.float32, device=self.dev)
        chunk = log_every if log_every else steps
        hist = []
        done = 0
        while done < steps:
            k = min(chunk, steps - done)
            # one cosine over the whole fit: each chunk covers its slice of the schedule
            f0, f1 = done / max(steps - 1, 1), (done + k - 1) / max(steps - 1, 1)
            l0 = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * f0))
            l1 = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * f1))
            _check(_lib.bp_surrogate_train(_ptr(self.w), _ptr(self.wb), _ptr(self.m), _ptr(self.v), _ptr(self.g),
                                           _ptr(self.mean), _ptr(self.std), n, _ptr(x), _ptr(t), k, batch,
                                           float(l0), float(l1), int(seed) & 0xFFFFFFFFFFFFFFFF, self.step,
                                           _ptr(loss), _ptr(ws), ws.numel(), _stream()), "bp_surrogate_train")
            self.step += k
            done += k
            if log_every:
                hist.append((done, float(loss.sum().item()) / (batch * 176)))
        return hist

    # -- inference -------------------------------------------------------------
    def infer(self, M, c, z, tables="exact"):
        """Network outputs, then the ICM solve seeded by the network's x_f (bp_surrogate_solve) and the
        q-tables: tables="exact" integrates the solved profiles at the 64 q nodes
        (bp_surrogate_qtables_exact); tables="network" takes the network's own table outputs
        (bp_surrogate_apply).  Returns sol, status (non-zero where the exact path must be used: outside
        the training domain or no root near the estimate), q-tables [n, 128], meta."""
        if tables not in ("exact", "network"):
            raise ValueError(f"tables must be 'exact' or 'network', not {tables!r}")
        n = M.numel()
        x = self.features(M, c, z)
        y = self.predict(x)
        sol, st = surrogate_solve(self.params, M, c, z, y, self.mean, self.std)
        qt = torch.zeros((n, 2 * MLP_NQ), dtype=torch.float32, device=self.dev)
        meta = torch.zeros((META_NFIELDS, n), dtype=torch.float32, device=self.dev)
        if tables == "exact":
            _check(_lib.bp_surrogate_qtables_exact(C.byref(self.params), n, _ptr(sol), _ptr(st), _ptr(qt), _ptr(meta),
                                                   _stream()), "bp_surrogate_qtables_exact")
        else:
            _check(_lib.bp_surrogate_apply(C.byref(self.params), n, _ptr(y), _ptr(self.mean), _ptr(self.std),
                                           _ptr(sol), _ptr(st), _ptr(qt), _ptr(meta), _stream()), "bp_surrogate_apply")
        return sol, st, qt, meta

    def fit_exact(self, M, c, z, steps, batch=4096, lr=2e-3, lr_end=1e-5, seed=0, ws: Workspace | None = None):
        """Training in one library call (bp_surrogate_fit): exact solves, tables, targets and statistics of the
        n halos (M, c, z device tensors), then Adam."""
        ws = ws or _ws_for(self.dev)
        _with_workspace(_lib.bp_surrogate_fit, "bp_surrogate_fit", ws,
                        (C.byref(self.params), _ptr(self.state), M.numel(), _ptr(M), _ptr(c), _ptr(z), int(steps),
                         int(batch), float(lr), float(lr_end), int(seed) & 0xFFFFFFFFFFFFFFFF, self.step))
        self.step += int(steps)

    def paste_healpix(self, cat_dev, nside, y_map, b_map, ws: Workspace | None = None, tables="exact", comp=None):
        """Surrogate HP paste onto HEALPix RING maps (bp_surrogate_paste_healpix: routing, the fallback's exact
        solve and the deposit on the device).  cat_dev holds M, c, z, theta, phi, v_los; comp = (y_comp, b_comp)
        carries the Kahan compensation.  Returns the number of halos routed to the exact solve."""
        ws = ws or _ws_for(y_map.device)
        nout = C.c_int64(0)
        d = cat_dev
        _with_workspace(_lib.bp_surrogate_paste_healpix, "bp_surrogate_paste_healpix", ws,
                        (C.byref(self.params), _ptr(self.state), SUR_TABLES[tables], int(nside), d["M"].numel(),
                         _ptr(d["M"]), _ptr(d["c"]), _ptr(d["z"]), _ptr(d["theta"]), _ptr(d["phi"]), _ptr(d["v_los"]),
                         _ptr(y_map), _ptr(b_map), *_comp_ptrs(comp, y_map)), tail=(C.byref(nout),))
        return nout.value

    def paste_flat(self, cat_dev, npix, pix_rad, y_map, b_map, ws: Workspace | None = None, tables="exact", comp=None):
        """Surrogate HP paste onto a flat map (bp_surrogate_paste_flat).  Returns the number of halos routed to
        the exact solve."""
        ws = ws or _ws_for(y_map.device)
        nout = C.c_int64(0)
        d = cat_dev
        _with_workspace(_lib.bp_surrogate_paste_flat, "bp_surrogate_paste_flat", ws,
                        (C.byref(self.params), _ptr(self.state), SUR_TABLES[tables], int(npix), float(pix_rad),
                         d["M"].numel(), _ptr(d["M"]), _ptr(d["c"]), _ptr(d["z"]), _ptr(d["theta_x"]),
                         _ptr(d["theta_y"]), _ptr(d["v_los"]), _ptr(y_map), _ptr(b_map), *_comp_ptrs(comp, y_map)),
                        tail=(C.byref(nout),))
        return nout.value
