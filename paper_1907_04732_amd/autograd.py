"""torch.autograd entry to the reverse mode of liblbe (lbe_record /
lbe_adjoint): the electrode charges and the total fluid momentum (under an
applied field, the electro-osmotic flux) after a number of time steps as
differentiable functions of the electrode potentials, the Bjerrum length and
the initial state.  Marshalling only: the forward steps, the checkpoints, the
recomputation and the reverse sweep all run in the library.

Tensors live on the host (the library copies them to the device); the
result is float64.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Lbe, make_params


class ElectrodeCharge(torch.autograd.Function):
    """(Q(T), M(T)) from (phi_s, l_B, n_init, f_init): one charge per
    electrode and the three components of the total fluid momentum
    sum_r (sum_i f_i c_i + F/2).

    `setup` holds the fixed inputs: shape, node_type, nsteps, every (the
    checkpoint interval) and the remaining keyword arguments of make_params
    (FP64 form).  each backward() call runs lbe_adjoint with the incoming weights.
    """

    @staticmethod
    def forward(ctx, phi_s, lB, n_init, f_init, setup):
        kw = dict(setup["params"])
        p = make_params(setup["shape"], lB=float(lB), **kw)
        as_np = lambda x: x.detach().cpu().double().numpy()  # noqa: E731
        sim = Lbe(p, setup["node_type"], as_np(phi_s), n_init=as_np(n_init), f_init=as_np(f_init))
        sim.record(setup["nsteps"], setup.get("every", 64))
        ctx.sim = sim
        ctx.shapes = (phi_s.shape, n_init.shape, f_init.shape)
        mom = np.array(sim.totals()["momentum"])
        return torch.from_numpy(sim.qhist()[-1].copy()), torch.from_numpy(mom)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, gq, gm):
        sim = ctx.sim
        want = ctx.needs_input_grad
        # the record stays valid: backward may run more than once (its device
        # memory goes with the graph)
        g = sim.adjoint(gq.detach().cpu().double().numpy(), gm.detach().cpu().double().numpy(),
                        phi_s=want[0], lB=want[1], n=want[2], f=want[3])
        s_phi, s_n, s_f = ctx.shapes
        out_phi = torch.from_numpy(g["phi_s"]).reshape(s_phi) if want[0] else None
        out_lb = torch.tensor(g["lB"], dtype=torch.float64) if want[1] else None
        out_n = torch.from_numpy(np.ascontiguousarray(g["n"])).reshape(s_n) if want[2] else None
        out_f = torch.from_numpy(np.ascontiguousarray(g["f"])).reshape(s_f) if want[3] else None
        return out_phi, out_lb, out_n, out_f, None


def charge_and_momentum(phi_s, lB, n_init, f_init, *, shape, node_type, nsteps, every=64,
                        **params):
    """(Q_e, M) after `nsteps` steps; differentiable in every tensor argument."""
    setup = dict(shape=tuple(shape), node_type=np.asarray(node_type), nsteps=int(nsteps),
                 every=int(every), params=params)
    return ElectrodeCharge.apply(phi_s, lB, n_init, f_init, setup)


def electrode_charge(phi_s, lB, n_init, f_init, **kw):
    """Q_e after `nsteps` steps; differentiable in every tensor argument."""
    return charge_and_momentum(phi_s, lB, n_init, f_init, **kw)[0]
