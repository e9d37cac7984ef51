"""Discrete velocity sets and the raw-moment basis (oracle; test infrastructure only).

Velocity set: the paper prints D3Q19 weights (1/3, 1/18, 1/36) next to Eq. 16
while calling the model D3Q17; the weights decide it: D3Q19 in 3D.  The 2D
workloads use D2Q9 (weights 4/9, 1/9, 1/36).  c_s^2 = 1/3 (text after Eq. 16).

Moment basis (Eq. 15, "simplified non-orthogonal" raw moments; the exact set of
the cited references is not in the paper): plain monomials e_x^a e_y^b e_z^c,
D2Q9 {1, x, y, x2, y2, xy, x2y, xy2, x2y2}; D3Q19 {1, x, y, z, x2, y2, z2, xy,
xz, yz, x2y, x2z, xy2, y2z, xz2, yz2, x2y2, x2z2, y2z2}.  M[k, n] is monomial k
evaluated at e_n; M^-1 comes from a library inverse.

Canonical direction order (it fixes tie-breaks of the wetting-link rule):
D2Q9  0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)
D3Q19 0:rest, 1..6: +x -x +y -y +z -z, 7..18: (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0)
      (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
"""
import torch

F64 = torch.float64


class Lattice:
    def __init__(self, dim: int):
        if dim == 2:
            e = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
                 (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)]
            w = [4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4
            mono = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (2, 0, 0), (0, 2, 0), (1, 1, 0),
                    (2, 1, 0), (1, 2, 0), (2, 2, 0)]
        elif dim == 3:
            e = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
                 (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
                 (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
                 (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
            w = [1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12
            mono = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (0, 2, 0), (0, 0, 2),
                    (1, 1, 0), (1, 0, 1), (0, 1, 1), (2, 1, 0), (2, 0, 1), (1, 2, 0), (0, 2, 1),
                    (1, 0, 2), (0, 1, 2), (2, 2, 0), (2, 0, 2), (0, 2, 2)]
        else:
            raise ValueError("dim must be 2 or 3")
        self.dim = dim
        self.Q = len(e)
        self.e_int = e
        self.e = torch.tensor(e, dtype=F64)                 # (Q, 3)
        self.w = torch.tensor(w, dtype=F64)                 # (Q,)
        self.cs2 = 1.0 / 3.0
        self.opp = [e.index(tuple(-c for c in v)) for v in e]
        self.mono = mono
        self.order = [sum(p) for p in mono]
        M = torch.empty(self.Q, self.Q, dtype=F64)
        for k, p in enumerate(mono):
            for n, v in enumerate(e):
                M[k, n] = float(v[0] ** p[0] * v[1] ** p[1] * v[2] ** p[2])
        self.M = M
        self.Minv = torch.linalg.inv(M)
        # axis directions +a / -a, a < dim, used by the finite-volume potential stencil
        self.axis_dirs = []
        for a in range(dim):
            plus = [0, 0, 0]
            plus[a] = 1
            minus = [0, 0, 0]
            minus[a] = -1
            self.axis_dirs.append((e.index(tuple(plus)), e.index(tuple(minus))))
        self.length = torch.sqrt((self.e ** 2).sum(1))       # |e_n|
