"""Helpers shared by the GPU tests: run the HIP path and the oracle on the same inputs."""
import numpy as np
import torch

from oracle import Oracle

FIELD_MAP = dict(phi1=("phi", 0), phi2=("phi", 1), phi3=("phi", 2), ux=("u", 0), uy=("u", 1), uz=("u", 2),
                 p=("p", None), rho_e=("rho_e", None))


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
    from paper_2608_12868_amd import _lib
    _lib.lib()   # raises if libehdlb.so is missing: no fallback


def oracle_run(case, steps, params=None, rho0=None, volts_fn=None):
    p = dict(case.params)
    if params:
        p.update(params)
    o = Oracle(case.dim, case.n, case.periodic, p, case.flags)
    s = o.init_state(case.phi, rho0)
    aux = None
    for _ in range(steps):
        v = volts_fn(s.t) if volts_fn else None
        s, aux = o.step(s, v)
    return o, s, aux


def oracle_fields(o, s, aux):
    f = o.fields(s)
    out = {}
    for k, (name, i) in FIELD_MAP.items():
        if name == "u" and i >= o.lat.dim:
            continue
        v = f[name] if i is None else f[name][i]
        out[k] = v.detach().numpy()
    if aux is not None and "pot" in aux:
        out["pot"] = aux["pot"].detach().numpy()
        out["q"] = (aux["Q"]).detach().numpy()
    return out


def rel_err(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def oracle_pops(o, s):
    """Oracle populations in the library's canonical order [family][q][node]."""
    parts = [s.g, s.f[0], s.f[1], s.f[2]]
    if o.ehd:
        parts.append(s.h)
    return torch.cat([p.reshape(-1) for p in parts]).detach().numpy()
