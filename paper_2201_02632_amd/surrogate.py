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

from . import (MLP_IN, MLP_OUT, S_OUT_OF_DOMAIN, SOL_NFIELDS, META_NFIELDS, MLP_NQ, _check, _lib, _ptr, _stream,
               Workspace, default_params, hp_paste_flat, hp_paste_flat_q, hp_paste_healpix, hp_paste_healpix_q,
               icm_solve, profile_tables, surrogate_solve)


def _f64(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


class Surrogate:
    """MLP (3 -> 256 -> 256 -> 256 -> 144) with FP32 master weights, a BF16
    compute copy and Adam state, all device-resident."""

    def __init__(self, params=None, device="cuda", seed=0):
        self.params = params or default_params()
        self.dev = torch.device(device)
        self.np = int(_lib.bp_mlp_nparams())
        self.w = torch.zeros(self.np, dtype=torch.float32, device=self.dev)
        self.wb = torch.zeros(self.np, dtype=torch.int16, device=self.dev)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.g = torch.zeros_like(self.w)
        self.mean = torch.zeros(MLP_OUT, dtype=torch.float32, device=self.dev)
        self.std = torch.ones(MLP_OUT, dtype=torch.float32, device=self.dev)
        self.step = 0
        self._init_weights(seed)

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

    def _init_weights(self, seed):
        """He-style initial weights from a seeded generator (an input to the method, like any data)."""
        rng = np.random.default_rng(seed)
        w = np.zeros(self.np, dtype=np.float32)
        L = self._layout()
        fan = {"W1": 3, "W2": 256, "W3": 256, "W4": 256}
        for name in ("W1", "W2", "W3", "W4"):
            off, n = L[name]
            block = rng.normal(0.0, math.sqrt(2.0 / fan[name]), size=n).astype(np.float32)
            if name == "W1":
                block = block.reshape(256, MLP_IN)
                block[:, 3:] = 0.0
                block = block.ravel()
            w[off:off + n] = block
        self.w.copy_(torch.from_numpy(w))
        _check(_lib.bp_mlp_to_bf16(self.np, _ptr(self.w), _ptr(self.wb), _stream()), "bp_mlp_to_bf16")

    def state_dict(self):
        return {"w": self.w.cpu().numpy(), "mean": self.mean.cpu().numpy(), "std": self.std.cpu().numpy(),
                "m": self.m.cpu().numpy(), "v": self.v.cpu().numpy(), "step": np.array(self.step)}

    def save(self, path):
        np.savez(path, **self.state_dict())

    def load(self, path):
        d = np.load(path, allow_pickle=False)
        self.w.copy_(torch.from_numpy(d["w"]))
        self.mean.copy_(torch.from_numpy(d["mean"]))
        self.std.copy_(torch.from_numpy(d["std"]))
        self.m.copy_(torch.from_numpy(d["m"]))
        self.v.copy_(torch.from_numpy(d["v"]))
        self.step = int(d["step"])
        _check(_lib.bp_mlp_to_bf16(self.np, _ptr(self.w), _ptr(self.wb), _stream()), "bp_mlp_to_bf16")

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

    def _fallback(self, cat_dev, st, paste):
        """Halos the network does not cover (non-zero status) through the exact solve and tables."""
        out = torch.nonzero(st != 0).flatten()
        nout = int(out.numel())
        if nout:
            sub = {k: v.index_select(0, out).contiguous() for k, v in cat_dev.items()}
            s2, st2 = icm_solve(self.params, sub["M"], sub["c"], sub["z"])
            tb2, mt2 = profile_tables(self.params, s2, st2)
            paste(sub, s2, st2, tb2, mt2)
        return nout

    def paste_healpix(self, cat_dev, nside, y_map, b_map, ws: Workspace | None = None, tables="exact", comp=None):
        """Surrogate HP paste onto HEALPix RING maps, exact fallback for halos outside the training domain.
        cat_dev holds M, c, z, theta, phi, v_los; comp = (y_comp, b_comp) carries the Kahan compensation."""
        sol, st, qt, meta = self.infer(cat_dev["M"], cat_dev["c"], cat_dev["z"], tables)
        hp_paste_healpix_q(self.params, nside, cat_dev["theta"], cat_dev["phi"], cat_dev["v_los"], sol, st, qt, meta,
                           y_map, b_map, ws, comp)
        del sol, qt, meta
        return self._fallback(cat_dev, st, lambda sub, s2, st2, tb2, mt2: hp_paste_healpix(
            self.params, nside, sub["theta"], sub["phi"], sub["v_los"], s2, st2, tb2, mt2, y_map, b_map, ws, comp))

    def paste_flat(self, cat_dev, npix, pix_rad, y_map, b_map, ws: Workspace | None = None, tables="exact", comp=None):
        """Surrogate HP paste with exact fallback for halos outside the training domain."""
        sol, st, qt, meta = self.infer(cat_dev["M"], cat_dev["c"], cat_dev["z"], tables)
        hp_paste_flat_q(self.params, npix, pix_rad, cat_dev["theta_x"], cat_dev["theta_y"], cat_dev["v_los"], sol,
                        st, qt, meta, y_map, b_map, ws, comp)
        del sol, qt, meta
        return self._fallback(cat_dev, st, lambda sub, s2, st2, tb2, mt2: hp_paste_flat(
            self.params, npix, pix_rad, sub["theta_x"], sub["theta_y"], sub["v_los"], s2, st2, tb2, mt2, y_map, b_map,
            ws, comp))
