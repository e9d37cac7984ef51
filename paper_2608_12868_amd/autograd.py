"""torch.autograd boundary of the hand-written adjoint.

ScheduleToObservables maps a piecewise-constant voltage schedule of one
electrode to the droplet's centroid and velocity after T steps; its backward
runs the library's checkpointed adjoint (recompute every K steps).
"""
import numpy as np
import torch


class ScheduleToObservables(torch.autograd.Function):
    @staticmethod
    def forward(ctx, volts, sim, phi0, T, K, t_total, electrode=0):
        v = volts.detach().to("cpu", torch.float64).numpy()
        sim.set_phase(phi0)
        sim.set_schedule(electrode, v, t_total)
        sim.forward_checkpointed(T, K)
        ob = sim.observables()
        ctx.sim, ctx.electrode, ctx.n_seg = sim, electrode, v.size
        ctx.generation = sim.generation
        return (torch.tensor(ob["centroid"], dtype=torch.float64),
                torch.tensor(ob["velocity"], dtype=torch.float64))

    @staticmethod
    def backward(ctx, g_centroid, g_velocity):
        gx = np.zeros(3) if g_centroid is None else g_centroid.detach().cpu().double().numpy()
        gv = np.zeros(3) if g_velocity is None else g_velocity.detach().cpu().double().numpy()
        if ctx.sim.generation != ctx.generation:
            raise RuntimeError("the simulation was changed or run again after this forward: its "
                               "checkpoints no longer belong to this graph node")
        g = ctx.sim.adjoint(gx, gv, ctx.electrode, ctx.n_seg)
        return torch.from_numpy(g), None, None, None, None, None, None


def schedule_to_observables(volts, sim, phi0, T, K, t_total, electrode=0):
    return ScheduleToObservables.apply(volts, sim, phi0, T, K, t_total, electrode)
