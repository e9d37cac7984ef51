"""FP64 CPU adjoint of the step (oracle; test infrastructure only).

The gradient of droplet observables at step T with respect to a piecewise-
constant electrode-voltage schedule is obtained by reverse-mode automatic
differentiation through the oracle's own steps: every operation of the step
is a differentiable torch op, and the exact potential solve carries its
adjoint (a solve with the same symmetric matrix).  Nothing here is hand-
derived; it is the plain definition of the discrete gradient.
"""
import torch

F64 = torch.float64


def segment_of(t, n_seg, t_total):
    """Schedule segment of step t: floor(t n_seg / t_total), clamped to the last segment."""
    return min(t * n_seg // t_total, n_seg - 1)


def observables_after(oracle, phi0, volts_seg, T, t_total, electrode=0, rho0=None):
    """Run T steps from the initial phase fields with electrode `electrode` driven by the
    schedule volts_seg (a tensor that may require grad); return (centroid, velocity) at T
    as differentiable tensors (the same definitions as Oracle.observables)."""
    s = oracle.init_state(phi0, rho0)
    base = torch.tensor(oracle.p["electrode_volts"], dtype=F64)
    n_seg = volts_seg.numel()
    for t in range(T):
        seg = segment_of(t, n_seg, t_total)
        sel = torch.zeros(base.numel(), dtype=torch.bool)
        sel[electrode] = True
        volts = torch.where(sel, volts_seg[seg], base)   # (NaN: a floating electrode)
        s, _ = oracle.step(s, volts)
    ob = oracle.observables(s)
    return ob["centroid"], ob["velocity"]


def schedule_gradient(oracle, phi0, volts_seg, T, t_total, dL_dxc, dL_dvc, electrode=0):
    """dL/dV per segment for L = dL_dxc . x_c(T) + dL_dvc . v_c(T) (a linearised loss: the
    caller's chain rule supplies the two cotangents)."""
    v = torch.as_tensor(volts_seg, dtype=F64).clone().requires_grad_(True)
    xc, vc = observables_after(oracle, phi0, v, T, t_total, electrode)
    L = (torch.as_tensor(dL_dxc, dtype=F64) * xc).sum() + (torch.as_tensor(dL_dvc, dtype=F64) * vc).sum()
    L.backward()
    return v.grad.detach().clone(), xc.detach(), vc.detach()
