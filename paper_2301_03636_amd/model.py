"""Owning wrapper of a libadvisor model handle."""
from __future__ import annotations

import numpy as np

from . import _lib


class Model:
    """A cost model (32 -> hidden widths -> 1) living on the current GPU."""

    def __init__(self, widths, precision="fp32"):
        self.widths = tuple(int(w) for w in widths)
        self.precision = precision
        self.handle = _lib.advisor_model_create(self.widths, precision)

    @property
    def param_count(self) -> int:
        return _lib.advisor_model_param_count(self.handle)

    def set_params(self, w_master, mu, sigma):
        _lib.advisor_model_set_params(self.handle, w_master, mu, sigma)

    def get_params(self):
        return _lib.advisor_model_get_params(self.handle)

    def set_zscore(self, mu, sigma):
        _lib.advisor_model_set_zscore(self.handle, mu, sigma)

    def calibrate_fp8(self, feat):
        _lib.advisor_model_calibrate_fp8(self.handle, feat)

    def fp8_scales(self):
        return _lib.advisor_model_get_fp8_scales(self.handle, len(self.widths) - 2)

    def predict(self, feat, pred_out=None):
        return _lib.advisor_predict(self.handle, feat, pred_out)

    def rank(self, kdesc, vdesc, offsets, best_out=None, pred_out=None, want_pred=False):
        return _lib.advisor_rank(self.handle, kdesc, vdesc, offsets, best_out, pred_out, want_pred)

    def rank_topn(self, kdesc, vdesc, offsets, top_n=10, idx_out=None, val_out=None, pred_out=None):
        """Each kernel's top_n variants by predicted runtime (the paper keeps
        N of them) and their predictions: (idx, val), each [n_kernels, top_n]."""
        return _lib.advisor_rank_topn(self.handle, kdesc, vdesc, offsets, top_n, idx_out, val_out,
                                      pred_out)

    def rank_refined(self, refine, kdesc, vdesc, offsets, top_k=8, best_out=None, pred_out=None):
        """Rank with this model, then re-rank each kernel's top_k candidates
        with `refine` (e.g. an fp32 model of the same weights)."""
        return _lib.advisor_rank_refined(self.handle, refine.handle, kdesc, vdesc, offsets, top_k,
                                         best_out, pred_out)

    def rank_cascade(self, later, keep, kdesc, vdesc, offsets, best_out=None, pred_out=None):
        """Rank with this model, hand each kernel's keep[0] best candidates
        to later[0], its keep[1] best to later[1], ...; the last model's
        argmin over its candidates is the pick (advisor_rank_cascade)."""
        return _lib.advisor_rank_cascade([self.handle] + [m.handle for m in later], keep, kdesc,
                                         vdesc, offsets, best_out, pred_out)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.advisor_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Plan:
    """A captured advisor_rank or advisor_train_step call (a HIP graph);
    launch() replays it on torch's current stream. Keep the model and every
    buffer named at creation alive while the plan exists."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    @classmethod
    def rank(cls, model, kdesc, vdesc, offsets, best_out, pred_out=None):
        h = _lib.advisor_rank_plan_create(model.handle, kdesc, vdesc, offsets, best_out, pred_out)
        return cls(h, (model, kdesc, vdesc, offsets, best_out, pred_out))

    @classmethod
    def train(cls, model, feat, y, loss_out, gnorm_out, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        h = _lib.advisor_train_plan_create(model.handle, feat, y, loss_out, gnorm_out, lr, beta1,
                                           beta2, eps)
        return cls(h, (model, feat, y, loss_out, gnorm_out))

    @classmethod
    def train_rmsprop(cls, model, feat, y, loss_out, gnorm_out, lr=1e-2, alpha=0.99, eps=1e-8,
                      weight_decay=1e-4, loss="rmse"):
        h = _lib.advisor_train_plan_create_rmsprop(model.handle, feat, y, loss_out, gnorm_out, lr,
                                                   alpha, eps, weight_decay, loss)
        return cls(h, (model, feat, y, loss_out, gnorm_out))

    @classmethod
    def train_rmsprop_multi(cls, models, feats, ys, loss_out=None, gnorm_out=None, lr=1e-2,
                            alpha=0.99, eps=1e-8, weight_decay=1e-4, loss="rmse"):
        """One RMSprop step of every model on its own batch, as one plan."""
        h = _lib.advisor_train_plan_create_rmsprop_multi([m.handle for m in models], feats, ys,
                                                         loss_out, gnorm_out, lr, alpha, eps,
                                                         weight_decay, loss)
        return cls(h, (list(models), list(feats), list(ys), loss_out, gnorm_out))

    def launch(self):
        _lib.advisor_plan_launch(self.handle)

    def rank_cascade(self, later, keep, kdesc, vdesc, offsets, best_out=None, pred_out=None):
        """Rank with this model, hand each kernel's keep[0] best candidates
        to later[0], its keep[1] best to later[1], ...; the last model's
        argmin over its candidates is the pick (advisor_rank_cascade)."""
        return _lib.advisor_rank_cascade([self.handle] + [m.handle for m in later], keep, kdesc,
                                         vdesc, offsets, best_out, pred_out)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.advisor_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def flops_per_variant(widths) -> int:
    """Algorithmic multiply-add flops of one forward pass (2 per MAC)."""
    return int(sum(2 * widths[i] * widths[i + 1] for i in range(len(widths) - 1)))


def as_numpy_params(w):
    return np.ascontiguousarray(w, dtype=np.float32)
