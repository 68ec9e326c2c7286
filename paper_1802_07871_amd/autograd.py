"""torch.autograd binding of the parameter adjoint (ctbop_param_grad).

    E, F, q = ctbop_efq(theta, pos, types, box, pbc, pot)
    loss = ((F - F_ref) ** 2).sum()
    loss.backward()              # theta.grad = dL/dtheta from the HIP adjoint

theta is a float64 tensor of the 56 parameters (any device; it is copied to
the context on every forward).  Each call evaluates the configuration in its
own system buffer, kept for the backward; gradients flow to theta only
(positions are data here).  Forward and backward run in the library's
kernels; this module marshals the seeds.
"""
from __future__ import annotations

import numpy as np

from . import System, _torch


class CTBOPFunction:
    """Namespace for the autograd.Function (built lazily so that importing the
    package does not import torch)."""
    _fn = None

    @classmethod
    def get(cls):
        if cls._fn is None:
            torch = _torch()

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(ctx, theta, pos, types, box, pbc, pot, Q):
                    th = theta.detach().to("cpu", torch.float64).numpy()
                    if not np.array_equal(th, pot.params):
                        pot.set_params(th)
                    n = types.shape[0]
                    s = System(pot, n, box, pbc)
                    pos_soa = pos.detach().to("cuda", torch.float64).reshape(-1, 3).t().contiguous().reshape(-1)
                    ty = types.to("cuda", torch.int32).contiguous()
                    E, F, q, _ = pot.compute_soa(pos_soa, ty, box, pbc, Q, warm=False, sysbuf=s, want_info=True)
                    ctx.state = (pot, s, box, pbc, n, theta.device, pot.params.copy())
                    return E.reshape(()), F.reshape(3, n).t().contiguous(), q

                @staticmethod
                def backward(ctx, gE, gF, gq):
                    pot, s, box, pbc, n, dev, th = ctx.state
                    if not np.array_equal(th, pot.params):
                        raise RuntimeError("the potential's parameters changed between forward and backward")
                    w = float(gE.item()) if gE is not None else 0.0
                    if gF is None:
                        gF = torch.zeros(n, 3, dtype=torch.float64, device="cuda")
                    vF = gF.to("cuda", torch.float64).t().contiguous().reshape(-1)
                    vq = gq.to("cuda", torch.float64).contiguous() if gq is not None else None
                    g, _ = pot.param_grad(s, box, pbc, w, vF, vq)
                    ctx.state = None
                    return torch.as_tensor(g, dtype=torch.float64, device=dev), None, None, None, None, None, None

            cls._fn = _F
        return cls._fn


def ctbop_efq(theta, pos, types, box, pbc, pot, Q: float = 0.0):
    """Differentiable (in theta) energy, forces (n,3) and charges (n,)."""
    torch = _torch()
    if torch.is_tensor(pos) and pos.requires_grad:
        raise NotImplementedError("gradients with respect to positions are not provided")
    pos = torch.as_tensor(pos, dtype=torch.float64)
    types = torch.as_tensor(np.asarray(types), dtype=torch.int32) if not torch.is_tensor(types) else types
    return CTBOPFunction.get().apply(theta, pos, types, box, pbc, pot, float(Q))
