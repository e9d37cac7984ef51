"""Node classification, neighbour tables and wetting links (oracle; test infrastructure only).

Every axis wraps in index space; an axis that is not periodic must have solid
end layers, so the wrap never connects fluid across it.

Wetting links (reading of Eq. 20a, which gives n.grad(Phi) at the solid but not
how to impose it on a lattice): every solid node s with at least one fluid
neighbour gets one link n* along which its ghost value is extrapolated.  With
N_s = sum over fluid neighbours of 36*w_n*e_n (exact integers), n* maximises
(e_n . N_s)/|e_n| over fluid neighbours with e_n . N_s > 0, ties going to the
lowest canonical index; if N_s = 0, n* is the first fluid neighbour in
canonical order.
"""
import numpy as np
import torch

FLUID, GROUND, NEUMANN, ELECTRODE0 = 0, 1, 2, 3


class Geometry:
    def __init__(self, lat, n, periodic, flags):
        self.lat = lat
        self.n = tuple(int(v) for v in n)
        nx, ny, nz = self.n
        self.N = nx * ny * nz
        flags = np.asarray(flags, dtype=np.uint8).reshape(-1)
        assert flags.size == self.N
        self.flags_np = flags
        self.flags = torch.from_numpy(flags.astype(np.int64))
        self.fluid_np = flags == FLUID
        self.fluid = torch.from_numpy(self.fluid_np)
        self.solid = ~self.fluid
        # coordinates
        idx = np.arange(self.N)
        x = idx % nx
        y = (idx // nx) % ny
        z = idx // (nx * ny)
        self.xyz_np = np.stack([x, y, z])
        self.xyz = torch.from_numpy(self.xyz_np.astype(np.float64))
        for a in range(3):
            if not periodic[a] and self.n[a] > 1:
                lo = self.xyz_np[a] == 0
                hi = self.xyz_np[a] == self.n[a] - 1
                assert not self.fluid_np[lo | hi].any(), "non-periodic axis needs solid end layers"
        # neighbour table: nbr[q, x] = index of x + e_q (wrapping)
        nb = np.empty((lat.Q, self.N), dtype=np.int64)
        for q, (ex, ey, ez) in enumerate(lat.e_int):
            xx = (x + ex) % nx
            yy = (y + ey) % ny
            zz = (z + ez) % nz
            nb[q] = xx + nx * (yy + ny * zz)
        self.nbr_np = nb
        self.nbr = torch.from_numpy(nb)
        self._wetting_links()

    def _wetting_links(self):
        lat = self.lat
        wint = [int(round(36.0 * float(v))) for v in lat.w]
        sol, dirs = [], []
        for s in np.nonzero(~self.fluid_np)[0]:
            fl = [q for q in range(1, lat.Q) if self.fluid_np[self.nbr_np[q, s]]]
            if not fl:
                continue
            ns = [0, 0, 0]
            for q in fl:
                for a in range(3):
                    ns[a] += wint[q] * lat.e_int[q][a]
            if ns == [0, 0, 0]:
                best = fl[0]
            else:
                best = None
                for q in fl:
                    d = sum(lat.e_int[q][a] * ns[a] for a in range(3))
                    if d <= 0:
                        continue
                    l2 = sum(c * c for c in lat.e_int[q])
                    if best is None:
                        best, bd, bl2 = q, d, l2
                    elif d * d * bl2 > bd * bd * l2:   # d/|e| strictly larger
                        best, bd, bl2 = q, d, l2
            sol.append(int(s))
            dirs.append(int(best))
        self.ghost_nodes_np = np.asarray(sol, dtype=np.int64)
        self.ghost_dirs_np = np.asarray(dirs, dtype=np.int64)
        self.ghost_nodes = torch.from_numpy(self.ghost_nodes_np)
        self.ghost_src = torch.from_numpy(self.nbr_np[self.ghost_dirs_np, self.ghost_nodes_np]
                                          if sol else np.zeros(0, dtype=np.int64))
        self.ghost_len = lat.length[torch.from_numpy(self.ghost_dirs_np)] if sol else torch.zeros(0, dtype=torch.float64)
