"""Level-set optimisation loop of the paper's results (Sec. 2.1, Sec. 2.3, Sec. 2.6): maximise an effective figure
of merit subject to equality constraints on the volume and a second effective property.

The loop only sequences the library's calls and keeps the scalar history; every field operation (the
homogenisation, the sensitivities, the chain rule to the level set, the Hilbertian extension and
projection of the velocity, the HJ step and the reinitialisation) runs in the library's kernels.

Per iteration q:
  1. reinitialise at the start and every `reinit_every` iterations (the paper: every five), by default
     with the subcell fix, which keeps the zero level set in place (the plain first-order scheme moves
     it by a fraction of h per call and erodes members a few elements thick);
  2. solve the cell problems; figures of merit from the effective tensors;
  3. for the objective and each constraint: its gradient with respect to the tensors, the backward
     pass to dJ/dphi (the volume's is the chain rule of 1/N^3), j = -dJ/dphi;
  4. the projected velocity (phz_hpm_velocity) with the constraints' relative violations;
  5. one HJ step.
It stops by the paper's rule (at q >= 10: the objective changed by less than 0.2 h relative to each of
the five previous iterations and every relative violation is below 1e-3) or after `max_iters`.

Step control (on by default; a reading, since the paper leaves it to its library): a factor tau in [0.05, 1] scales
the objective part of the velocity.  It halves when the largest relative violation is above 1e-3 and has
not fallen by 10% over the last five iterations, and otherwise grows by 1.1.  The objective's step moves the
interface by up to cfl h per iteration, and its second-order effect on the constraints does not fade
with a fixed step; the constraint part, first order, then holds them only at a nonzero violation.
"""
from __future__ import annotations

import time

import numpy as np

from . import PHZ_OK, foms

PROPERTIES = ("B_voigt", "B_reuss", "d_h", "g_h", "k_h", "C_zzzz", "vol")


def _value_and_tensor_grads(name, CH, eH, kH):
    """Value of an effective property and its gradient with respect to (C^H, e^H, kappa^H)."""
    if name == "C_zzzz":
        gC = np.zeros((6, 6))
        gC[2, 2] = 1.0
        return float(CH[2, 2]), (gC, np.zeros((3, 6)), np.zeros((3, 3)))
    f, grads = foms(CH, eH, kH, grad_of=name)
    return float(f[name]), grads


class _DeviceFields:
    """Node-sized device tensors of one optimisation (the sensitivities, the velocity and the level set
    stay on the device between the library's calls; only scalars come back to the host)."""

    def __init__(self, ctx, m):
        import torch
        self.torch = torch
        dev = torch.device("cuda", ctx.device)
        self.new = lambda: torch.empty(ctx.nn, dtype=torch.float64, device=dev)
        self.scale = self.new()
        self.grad_rho = self.new()
        self.const = torch.full((ctx.nn,), 1.0 / ctx.nn, dtype=torch.float64, device=dev)
        self.gphi = [self.new() for _ in range(m + 1)]
        self.v = self.new()
        self.phi = self.new()
        self.ready()

    def ready(self):
        """Wait for this thread's torch work on the fields: the library reads them on the context's
        stream, which need not be torch's."""
        self.torch.cuda.current_stream().synchronize()


def _sensitivity(ctx, name, CH, eH, kH, void_scale, dev=None, slot=0):
    """(value, dValue/dphi) of a property at the context's solved geometry; with device fields, dValue/dphi
    is a device tensor (dev.gphi[slot])."""
    n3 = ctx.nn
    if dev is not None:
        if name == "vol":
            ctx.scale(out=dev.scale)
            vol = (float(dev.scale.mean()) - void_scale) / (1.0 - void_scale)
            return vol, ctx.levelset_gradient(dev.const, out=dev.gphi[slot])
        val, (gC, ge, gk) = _value_and_tensor_grads(name, CH, eH, kH)
        ctx.backward(gC, ge, gk, out_rho=dev.grad_rho, out_phi=dev.gphi[slot])
        return val, dev.gphi[slot]
    if name == "vol":
        rho = (ctx.scale() - void_scale) / (1.0 - void_scale)
        return float(np.mean(rho)), ctx.levelset_gradient(np.full(n3, 1.0 / n3))
    val, (gC, ge, gk) = _value_and_tensor_grads(name, CH, eH, kH)
    _, gphi = ctx.backward(gC, ge, gk, want_phi=True)
    return val, gphi


def should_stop(J_hist, viol_hist, h):
    """The paper's stopping rule on the objective and relative-violation histories."""
    q = len(J_hist) - 1
    if q < 10:
        return False
    Jq = J_hist[q]
    if any(abs(Jq - J_hist[q - j]) >= 0.2 * h * abs(Jq) for j in range(1, 6)):
        return False
    return all(abs(c) < 1e-3 for c in viol_hist[q])


def optimise(ctx, material, phi0, objective, constraints, max_iters=200, cfl=0.5, gamma=0.5, alpha=0.0,
             reinit_every=5, reinit_steps=20, reinit_subcell=True, step_control=True, callback=None):
    """Maximise `objective` subject to [(property, target), ...] equality constraints from the level set
    phi0 (nodes, x fastest).  Returns a dict with the histories, the final level set, the effective
    tensors of the last solved geometry and the wall time of each phase in ms per iteration (every
    library call returns after its device work).  A context
    created with warm_start=1 starts each solve from the last iteration's solution."""
    if objective not in PROPERTIES or objective == "vol":
        raise ValueError(f"objective must be one of {PROPERTIES[:-1]}")
    for name, target in constraints:
        if name not in PROPERTIES or not target:
            raise ValueError(f"bad constraint {(name, target)}")
    h = 1.0 / ctx.n
    ctx.set_levelset(np.ascontiguousarray(phi0, dtype=np.float64).ravel())
    # on a GPU context the node fields stay on the device
    dev = _DeviceFields(ctx, len(constraints)) if ctx.device is not None else None
    hist = {"J": [], "constraints": [], "violations": [], "status": [], "iter_ms": [], "tau": []}
    tau = 1.0
    phases = {"reinit": 0.0, "solve": 0.0, "sensitivities": 0.0, "velocity": 0.0, "hj": 0.0}
    phi = None
    clock = time.perf_counter

    def lap(name, t0):
        t1 = clock()
        phases[name] += 1e3 * (t1 - t0)
        return t1

    for q in range(max_iters):
        t = t_iter = clock()
        if reinit_every and q % reinit_every == 0:
            ctx.reinit(reinit_steps, cfl, subcell=reinit_subcell, return_phi=False)
            t = lap("reinit", t)
        status = ctx.solve()
        CH, eH, kH = ctx.effective()
        t = lap("solve", t)
        J, dJ = _sensitivity(ctx, objective, CH, eH, kH, material.void_scale, dev, 0)
        vals, viol, jc = [], [], []
        for i, (name, target) in enumerate(constraints):
            val, dC = _sensitivity(ctx, name, CH, eH, kH, material.void_scale, dev, 1 + i)
            vals.append(val)
            viol.append((val - target) / abs(target))
            if dev is not None:
                dC.mul_(-1.0 / abs(target))
                jc.append(dC)
            else:
                jc.append(-dC / abs(target))
        t = lap("sensitivities", t)
        hist["J"].append(J)
        hist["constraints"].append(vals)
        hist["violations"].append(viol)
        hist["status"].append(status)
        hist["effective"] = (CH, eH, kH)
        if callback:
            callback(q, J, vals, viol)
        if should_stop(hist["J"], hist["violations"], h):
            hist["iter_ms"].append(1e3 * (clock() - t_iter))
            break
        if step_control and q >= 5:
            now = max(map(abs, viol), default=0.0)
            before = max(map(abs, hist["violations"][-6]), default=0.0)
            tau = max(0.05, 0.5 * tau) if now > 1e-3 and now > 0.9 * before else min(1.0, 1.1 * tau)
        hist["tau"].append(tau)
        if dev is not None:
            dJ.neg_()
            dev.ready()
            v = ctx.hpm_velocity(dJ, jc, viol, alpha=alpha, cfl=cfl, gamma=gamma, obj_weight=tau, out=dev.v)
            t = lap("velocity", t)
            ctx.hj_step(v, cfl=cfl, out=dev.phi)
            phi = dev.phi
        else:
            v = ctx.hpm_velocity(-dJ, jc, viol, alpha=alpha, cfl=cfl, gamma=gamma, obj_weight=tau)
            t = lap("velocity", t)
            phi = ctx.hj_step(v, cfl=cfl, return_phi=True)
        lap("hj", t)
        hist["iter_ms"].append(1e3 * (clock() - t_iter))
    hist["phase_ms"] = {k: v / max(len(hist["J"]), 1) for k, v in phases.items()}
    hist["phi"] = phi.cpu().numpy() if phi is not None and dev is not None else phi
    hist["iterations"] = len(hist["J"])
    hist["converged"] = should_stop(hist["J"], hist["violations"], h)
    return hist
