"""Training drivers: a torch.autograd.Function whose forward and backward
are the library's hand-written kernels, and a loop around the library's own
fused training step (forward, float64 loss, backward, float64 gradient norm,
Adam)."""
from __future__ import annotations

import torch

from . import _lib


class MLPFunction(torch.autograd.Function):
    """y_hat = network(params; feat). `params` is the flat fp32 master vector
    (the layout of advisor_model_set_params) on the GPU; gradients flow to it
    through advisor_mlp_backward. The model handle's weights are replaced by
    `params` on every forward call."""

    @staticmethod
    def forward(ctx, params, feat, model):
        _lib.advisor_model_load_params(model.handle, params.detach().contiguous())
        y, saved = _lib.advisor_mlp_forward(model.handle, feat)
        ctx.model = model
        ctx.saved_buf = saved
        ctx.n = feat.shape[0]
        return y

    @staticmethod
    def backward(ctx, dy):
        g = _lib.advisor_mlp_backward(ctx.model.handle, dy.contiguous().to(torch.float32),
                                      ctx.saved_buf, ctx.n)
        return g, None, None


def mlp(params, feat, model):
    return MLPFunction.apply(params, feat, model)


class Trainer:
    """Adam on the MSE of ln-runtime, one fused library step per batch."""

    def __init__(self, model, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.model = model
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps

    def step(self, feat, y, loss_out=None, gnorm_out=None):
        return _lib.advisor_train_step(self.model.handle, feat, y, self.lr, self.beta1, self.beta2,
                                       self.eps, loss_out, gnorm_out)
