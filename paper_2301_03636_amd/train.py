"""Training drivers: a torch.autograd.Function whose forward and backward
are the library's hand-written kernels, and a loop around the library's own
fused training step (forward, float64 loss, backward, float64 gradient norm,
Adam or RMSprop)."""
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


def step_lr(epoch, lr0=1e-2, gamma=0.1, every=30):
    """Section 5.3's learning-rate schedule (advisor_step_lr): lr0,
    multiplied by gamma after every `every` epochs."""
    return _lib.advisor_step_lr(epoch, lr0, gamma, every)


class RMSpropTrainer:
    """Section 5.3's recipe in the library's fused step: RMSprop with weight
    decay 1e-4 on the RMSE loss, the learning rate 0.01 stepped down by 10x
    every 30 epochs (call set_epoch at each epoch). alpha and eps, which the
    paper leaves unstated, default to 0.99 and 1e-8."""

    def __init__(self, model, lr0=1e-2, alpha=0.99, eps=1e-8, weight_decay=1e-4, loss="rmse",
                 gamma=0.1, every=30):
        self.model = model
        self.lr0, self.gamma, self.every = lr0, gamma, every
        self.alpha, self.eps, self.weight_decay, self.loss = alpha, eps, weight_decay, loss
        self.lr = lr0

    def set_epoch(self, epoch):
        self.lr = step_lr(epoch, self.lr0, self.gamma, self.every)

    def step(self, feat, y, loss_out=None, gnorm_out=None):
        return _lib.advisor_train_step_rmsprop(self.model.handle, feat, y, self.lr, self.alpha,
                                               self.eps, self.weight_decay, self.loss, loss_out,
                                               gnorm_out)
