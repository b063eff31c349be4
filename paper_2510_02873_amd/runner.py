"""Convenience wrapper around one pino_ctx (argument marshalling only)."""

from __future__ import annotations

import torch

from . import _abi


class Collapse:
    """One library context.  Outputs are caller-owned device tensors:
    Fmax float64, Rmax int32, a_coll float64 (optional)."""

    def __init__(self, growth_tables, method=_abi.PINO_CLASSIC, precision=_abi.PINO_FP64, device=0,
                 table_knots=None, mlp_blob=None, certify_rtol=0.0):
        self.device = torch.device("cuda", device)
        self.method = method
        self.precision = precision
        self._cfg = _abi.Config(growth_tables, method=method, precision=precision, device=device,
                                table_knots=table_knots, mlp_blob=mlp_blob, certify_rtol=certify_rtol)
        self.ctx = _abi.pino_collapse_init(self._cfg)

    def outputs(self, n):
        Fmax = torch.zeros(n, dtype=torch.float64, device=self.device)
        Rmax = torch.full((n,), -1, dtype=torch.int32, device=self.device)
        acoll = torch.full((n,), float("inf"), dtype=torch.float64, device=self.device)
        return Fmax, Rmax, acoll

    def item(self, h, Fmax, Rmax, acoll=None, radius_index=0, cosmo=0, sigma_R=1.0, table_F=None):
        want = torch.float32 if self.precision == _abi.PINO_MIXED else torch.float64
        for c in range(6):
            t = h[c]
            if t.dtype != want or not t.is_contiguous() or t.device != self.device:
                raise ValueError(f"Hessian component {c} must be a contiguous {want} tensor on {self.device}")
        n = h[0].numel()
        for t, dt in ((Fmax, torch.float64), (Rmax, torch.int32)):
            if t.dtype != dt or t.numel() != n or not t.is_contiguous() or t.device != self.device:
                raise ValueError("outputs must be contiguous device tensors of matching length")
        if acoll is not None and (acoll.dtype != torch.float64 or acoll.numel() != n or not acoll.is_contiguous()):
            raise ValueError("a_coll must be a contiguous float64 tensor of matching length")
        if table_F is not None and (table_F.dtype != torch.float64 or not table_F.is_contiguous()):
            raise ValueError("table_F must be a contiguous float64 device tensor")
        return _abi.make_item(h, Fmax, Rmax, acoll, radius_index=radius_index, cosmo=cosmo,
                              sigma_R=sigma_R, table_F=table_F)

    def eval(self, items, reset=False, sync=False, stream=None, finalize=False):
        flags = ((_abi.PINO_EVAL_RESET if reset else 0) | (_abi.PINO_EVAL_SYNC if sync else 0)
                 | (_abi.PINO_EVAL_FINALIZE if finalize else 0))
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        _abi.pino_collapse_eval(self.ctx, list(items), flags, stream)

    def apply(self, h, radius_index, Fmax, Rmax, acoll=None, reset=False, cosmo=0, sigma_R=1.0,
              table_F=None, sync=False, stream=None, finalize=False):
        self.eval([self.item(h, Fmax, Rmax, acoll, radius_index, cosmo, sigma_R, table_F)], reset=reset,
                  sync=sync, stream=stream, finalize=finalize)

    def close(self):
        if self.ctx is not None:
            _abi.pino_collapse_free(self.ctx)
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
