"""Python face of libehdlb: a Simulation owns one library context.

PyTorch provides the device workspace (one uint8 tensor) and the stream; every
step of the method runs in the library's HIP kernels.
"""
import ctypes as C
import weakref

import numpy as np

from . import _lib as L


def make_structs(dim, n, periodic, precision, params):
    lat = L.Lattice()
    lat.dim = int(dim)
    for a in range(3):
        lat.n[a] = int(n[a])
        lat.periodic[a] = int(periodic[a])
    lat.precision = L.FP64 if precision in ("fp64", L.FP64) else L.FP32_DEV
    p = L.Params()
    for i in range(3):
        p.tau_flow[i] = float(params["tau_flow"][i])
        p.eps[i] = float(params["eps"][i])
        p.cond[i] = float(params["cond"][i])
        p.body_force[i] = float(params["body_force"][i])
    for k in ("mobility", "width", "gamma12", "gamma13", "gamma23", "cos12", "cos13", "cos23",
              "charge_diffusion", "poisson_tol"):
        setattr(p, k, float(params[k]))
    p.ehd = int(params["ehd"])
    for k in range(L.MAX_ELECTRODES):
        p.electrode_volts[k] = float(params["electrode_volts"][k])
    p.poisson_max_iter = int(params["poisson_max_iter"])
    p.poisson_check_every = int(params["poisson_check_every"])
    p.s_high = float(params.get("s_high", 1.0))
    for i, v in enumerate(params.get("rho", (1.0, 1.0, 1.0))):
        p.rho[i] = float(v)
    return lat, p


def preset(name, seed=0):
    """The library's host-only workload preset: (lattice, params, flags, phi) as ctypes structs
    and numpy arrays (ehdlb_preset)."""
    pid = L.PRESETS[name]
    lat, p = L.Lattice(), L.Params()
    st = L.lib().ehdlb_preset(pid, C.byref(lat), C.byref(p), None, None, int(seed))
    if st != L.OK:
        raise L.EhdlbError(st, f"ehdlb_preset rejected {name}")
    N = lat.n[0] * lat.n[1] * lat.n[2]
    flags = np.zeros(N, np.uint8)
    phi = np.zeros((3, N), np.float64)
    L.lib().ehdlb_preset(pid, C.byref(lat), C.byref(p), flags.ctypes.data, phi.ctypes.data, int(seed))
    return lat, p, flags, phi


class Context:
    """A library context without device memory: validation and host-side tables only."""

    def __init__(self, dim, n, periodic, precision, params):
        self.dim, self.n = int(dim), tuple(int(v) for v in n)
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.precision = precision
        self.params = dict(params)
        lat, p = make_structs(dim, n, periodic, precision, params)
        h = C.c_void_p()
        st = L.lib().ehdlb_create(C.byref(lat), C.byref(p), C.byref(h))
        if st != L.OK:
            raise L.EhdlbError(st, "ehdlb_create rejected the lattice or parameters")
        self.h = h
        # destroy the context when this object is collected, or at interpreter exit while the
        # library and ctypes are still loaded (a __del__ could run after module teardown)
        self._finalizer = weakref.finalize(self, L.lib().ehdlb_destroy, h)

    def _chk(self, st):
        return L.check(self.h, st)

    def set_geometry(self, flags):
        self._flags = np.ascontiguousarray(flags, dtype=np.uint8).reshape(-1)
        if self._flags.size != self.N:
            raise ValueError("flags must have N entries")
        self._chk(L.lib().ehdlb_set_geometry(self.h, self._flags.ctypes.data))

    def wetting_links(self):
        n = L.lib().ehdlb_wetting_links(self.h, None, None, 0)
        if n < 0:
            self._chk(int(n))
        nodes = np.zeros(n, np.int64)
        dirs = np.zeros(n, np.int32)
        L.lib().ehdlb_wetting_links(self.h, nodes.ctypes.data, dirs.ctypes.data, n)
        return nodes, dirs

    @property
    def generation(self):
        """Counter bumped by every call that changes the state or the steps (ehdlb_generation)."""
        return int(L.lib().ehdlb_generation(self.h))

    @property
    def workspace_bytes(self):
        return int(L.lib().ehdlb_workspace_bytes(self.h))


class Simulation(Context):
    """A bound context: device workspace from torch, work on torch's current stream."""

    def __init__(self, dim, n, periodic, precision, params, flags, phi, device="cuda"):
        import torch
        super().__init__(dim, n, periodic, precision, params)
        self.torch = torch
        self.device = torch.device(device)
        nbytes = self.workspace_bytes
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.stream = torch.cuda.current_stream(self.device)
        self._chk(L.lib().ehdlb_bind(self.h, C.c_void_p(base + off), nbytes, C.c_void_p(self.stream.cuda_stream)))
        self.set_geometry(flags)
        self.set_phase(phi)

    @classmethod
    def from_case(cls, case, precision=None, **over):
        params = dict(case.params)
        params.update(over)
        return cls(case.dim, case.n, case.periodic, precision or case.precision, params, case.flags, case.phi)

    def set_phase(self, phi):
        a = np.ascontiguousarray(phi, dtype=np.float64).reshape(3, self.N)
        self._chk(L.lib().ehdlb_set_phase(self.h, a.ctypes.data))

    def set_charge(self, rho):
        a = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.N)
        self._chk(L.lib().ehdlb_set_charge(self.h, a.ctypes.data))

    def set_schedule(self, electrode, volts, t_total):
        v = np.ascontiguousarray(volts, dtype=np.float64)
        self._chk(L.lib().ehdlb_set_schedule(self.h, int(electrode), int(v.size), v.ctypes.data, int(t_total)))

    def step(self, n=1):
        self._chk(L.lib().ehdlb_step(self.h, int(n)))

    def field(self, name, device=False):
        """One field as float64: a numpy array, or (device=True) a torch tensor on the
        simulation's device written by the library on its stream."""
        fid = L.FIELDS[name]
        size = int(L.lib().ehdlb_num_populations(self.h)) if name == "pops" else self.N
        if device:
            out = self.torch.empty(size, dtype=self.torch.float64, device=self.device)
            self._chk(L.lib().ehdlb_read_field(self.h, fid, C.c_void_p(out.data_ptr()), 1))
            return out
        out = np.empty(size, np.float64)
        self._chk(L.lib().ehdlb_read_field(self.h, fid, out.ctypes.data, 0))
        return out

    def observables(self, strict=True):
        o = L.Obs()
        st = L.lib().ehdlb_observables(self.h, C.byref(o))
        if strict:
            self._chk(st)
        return dict(step=o.step, mass=np.array(o.mass[:]), centroid=np.array(o.centroid[:]),
                    velocity=np.array(o.velocity[:]), total_charge=o.total_charge,
                    sum_phi_drift=o.sum_phi_drift, poisson_residual=o.poisson_residual,
                    poisson_initial_residual=o.poisson_initial_residual,
                    poisson_iters=o.poisson_iters, flags=o.flags, status=st)

    def adjoint_workspace_bytes(self, T, K):
        return int(L.lib().ehdlb_adjoint_workspace_bytes(self.h, int(T), int(K)))

    def forward_checkpointed(self, T, K):
        """Run T steps keeping a checkpoint every K steps (device memory owned by this object)."""
        torch = self.torch
        nbytes = self.adjoint_workspace_bytes(T, K)
        if getattr(self, "adj_ws", None) is None or self.adj_ws.numel() < nbytes + 256:
            self.adj_ws = None
            self.adj_ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.adj_ws.data_ptr()
        ptr = base + ((-base) % 256)
        self._chk(L.lib().ehdlb_forward_checkpointed(self.h, int(T), int(K), C.c_void_p(ptr), nbytes))

    def adjoint(self, dL_dcentroid, dL_dvelocity, electrode=0, n_seg=None):
        """dL/dV per schedule segment of `electrode` after forward_checkpointed."""
        gx = np.ascontiguousarray(dL_dcentroid, dtype=np.float64).reshape(3)
        gv = np.ascontiguousarray(dL_dvelocity, dtype=np.float64).reshape(3)
        out = np.zeros(max(int(n_seg or 1), 1), np.float64)
        self._chk(L.lib().ehdlb_adjoint(self.h, gx.ctypes.data, gv.ctypes.data, int(electrode), out.ctypes.data))
        return out

    def solver_stats(self, reset=False):
        """Potential-solve statistics per kind (forward steps, adjoint): solves, CG iterations,
        largest initial relative residual."""
        counts = np.zeros(4, dtype=np.int64)
        rel0 = np.zeros(2)
        self._chk(L.lib().ehdlb_solver_stats(self.h, 1 if reset else 0, counts.ctypes.data, rel0.ctypes.data))
        return {k: dict(solves=int(counts[2 * j]), iters=int(counts[2 * j + 1]), max_rel0=float(rel0[j]))
                for j, k in enumerate(("forward", "adjoint"))}

    def set_solver_options(self, lo=0.5, hi=2.0, overcorrect=2.0, warm_start=4):
        """Chebyshev smoothing interval [lo, hi] of D^-1 A, coarse-correction scale, and the
        forward warm start (0: previous step's potential; 1: extrapolated from the last two;
        2: Galerkin projection onto the last five, then at least one CG iteration; 3: the
        projection alone; 4, the default: 3 in step(), 2 in forward_checkpointed() and the
        adjoint's recompute)."""
        self._chk(L.lib().ehdlb_set_solver_options(self.h, float(lo), float(hi), float(overcorrect),
                                                   int(warm_start)))

    def set_timing(self, on=True):
        self._chk(L.lib().ehdlb_set_timing(self.h, int(bool(on))))

    def timing(self):
        """(ms_moments, ms_potential, ms_step) summed over the timed steps, and their count."""
        ms = (C.c_double * 3)()
        n = C.c_int64()
        self._chk(L.lib().ehdlb_timing(self.h, ms, C.byref(n)))
        return list(ms), int(n.value)

    @property
    def state_bytes(self):
        return int(L.lib().ehdlb_state_bytes(self.h))

    def save_state(self, dst=None):
        torch = self.torch
        if dst is None:
            dst = torch.empty(self.state_bytes + 256, dtype=torch.uint8, device=self.device)
        ptr = dst.data_ptr() + ((-dst.data_ptr()) % 256)
        self._chk(L.lib().ehdlb_save_state(self.h, C.c_void_p(ptr)))
        return dst

    def load_state(self, src):
        ptr = src.data_ptr() + ((-src.data_ptr()) % 256)
        self._chk(L.lib().ehdlb_load_state(self.h, C.c_void_p(ptr)))
