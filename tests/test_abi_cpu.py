"""C ABI checks that need no GPU: the library loads, exports every declared symbol, validates
its inputs with the documented error codes, and builds the same wetting links as the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from inputs import make_case
from inputs.presets import ELECTRODE0, FLUID, GROUND, NEUMANN
from oracle.geometry import Geometry
from oracle.lattice import Lattice

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2608_12868_amd import _lib
    return _lib


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ehdlb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ehdlb_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(L):
    lib = C.CDLL(L.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding covers them all
    assert set(names) <= set(L.SIGNATURES)


def test_struct_layouts_match_header(L):
    assert C.sizeof(L.Lattice) == 32
    # 3 + 2 + 3 + 3 doubles, 2 ints, 3 + 3 + 1 + 3 + 4 + 1 doubles, 2 ints, 1 + 3 doubles
    assert C.sizeof(L.Params) == 8 * (3 + 2 + 3 + 3) + 8 + 8 * (3 + 3 + 1 + 3 + 4 + 1) + 8 + 8 * 4
    assert C.sizeof(L.Obs) == 8 + 8 * (3 + 3 + 3 + 4) + 8


def _ctx(case, **over):
    from paper_2608_12868_amd import Context
    p = dict(case.params)
    p.update(over)
    return Context(case.dim, case.n, case.periodic, case.precision, p)


@pytest.mark.parametrize("over", [dict(tau_flow=(0.5, 1, 1)), dict(mobility=0.0), dict(width=-1.0),
                                  dict(gamma12=1e-3, gamma13=2e-3, gamma23=1e-3), dict(gamma12=-1e-3),
                                  dict(eps=(80, 0, 1)),
                                  dict(cond=(-1, 0, 0)), dict(charge_diffusion=-1.0), dict(poisson_tol=0.0),
                                  dict(poisson_max_iter=0), dict(s_high=2.0), dict(s_high=-0.5),
                                  dict(rho=(1.0, 1.0, -2.0))])
def test_create_rejects_invalid_parameters(L, over):
    case = make_case("c2s")
    with pytest.raises(L.EhdlbError) as e:
        _ctx(case, **over)
    assert e.value.status == L.EINVAL


def test_create_rejects_bad_lattice(L):
    from paper_2608_12868_amd.sim import make_structs
    case = make_case("c1s")
    # bad dimension, 2D with Nz > 1, an empty axis, 2^31 nodes (the library takes fewer)
    for dim, n in ((4, case.n), (2, (16, 16, 2)), (3, (0, 4, 4)), (3, (2048, 1024, 1024))):
        lat, p = make_structs(dim, n, case.periodic, "fp64", case.params)
        h = C.c_void_p()
        assert L.lib().ehdlb_create(C.byref(lat), C.byref(p), C.byref(h)) == L.EINVAL


def test_geometry_validation(L):
    case = make_case("c2s")
    ctx = _ctx(case)
    ctx.set_geometry(case.flags)
    n = case.n
    # unknown flag
    bad = case.flags.copy()
    bad[100] = ELECTRODE0 + 7
    with pytest.raises(L.EhdlbError) as e:
        ctx.set_geometry(bad)
    assert e.value.status == L.EINVAL
    # fluid on the end layer of the non-periodic axis
    bad = case.flags.copy()
    bad[5] = FLUID
    with pytest.raises(L.EhdlbError):
        ctx.set_geometry(bad)
    # isolated fluid node
    bad = case.flags.copy()
    i = 20 * n[0] + 60
    bad[:] = np.where(np.isin(np.arange(bad.size), [i - 1, i + 1, i - n[0], i + n[0], i - n[0] - 1,
                                                     i - n[0] + 1, i + n[0] - 1, i + n[0] + 1]), NEUMANN, bad)
    with pytest.raises(L.EhdlbError):
        ctx.set_geometry(bad)
    # field on, but no grounded or electrode face anywhere
    bad = np.where(case.flags == FLUID, FLUID, NEUMANN).astype(np.uint8)
    with pytest.raises(L.EhdlbError):
        ctx.set_geometry(bad)


def test_calls_out_of_order(L):
    case = make_case("c1s")
    ctx = _ctx(case)
    assert L.lib().ehdlb_step(ctx.h, 1) == L.ESTATE
    obs = L.Obs()
    assert L.lib().ehdlb_observables(ctx.h, C.byref(obs)) == L.ESTATE
    out = np.zeros(case.N)
    assert L.lib().ehdlb_read_field(ctx.h, 0, out.ctypes.data, 0) == L.ESTATE
    assert L.lib().ehdlb_read_field(ctx.h, 0, out.ctypes.data, 2) == L.EINVAL
    assert L.lib().ehdlb_bind(ctx.h, C.c_void_p(0x1001), 10 ** 12, None) == L.EINVAL       # misaligned
    assert L.lib().ehdlb_bind(ctx.h, C.c_void_p(0x1000), 16, None) == L.ENOMEM             # too small
    assert L.lib().ehdlb_set_schedule(ctx.h, 9, 1, out.ctypes.data, 10) == L.EINVAL
    assert L.lib().ehdlb_set_solver_options(ctx.h, 0.5, 2.5, 2.0, 0) == L.EINVAL
    assert L.lib().ehdlb_set_solver_options(ctx.h, 0.5, 2.0, 2.0, 5) == L.EINVAL
    assert L.lib().ehdlb_set_solver_options(ctx.h, 0.5, 2.0, 2.0, 4) == L.OK


@pytest.mark.parametrize("name", ["c1s", "c2s", "c3s", "c2", "c3"])
def test_wetting_links_bit_exact_vs_oracle(name):
    """The library's host link table and the oracle's independent one agree bit for bit."""
    case = make_case(name)
    ctx = _ctx(case)
    ctx.set_geometry(case.flags)
    nodes, dirs = ctx.wetting_links()
    g = Geometry(Lattice(case.dim), case.n, case.periodic, case.flags)
    assert np.array_equal(nodes, g.ghost_nodes_np)
    assert np.array_equal(dirs, g.ghost_dirs_np)
    assert len(nodes) > 0


def test_workspace_sizes_scale(L):
    c32 = _ctx(make_case("c2s"), )
    from paper_2608_12868_amd import Context
    case = make_case("c2s")
    c64 = Context(case.dim, case.n, case.periodic, "fp64", case.params)
    c32 = Context(case.dim, case.n, case.periodic, "fp32", case.params)
    assert c32.workspace_bytes < c64.workspace_bytes
    per_node = c64.workspace_bytes / case.N
    assert 2 * 5 * 9 * 8 < per_node < 2000


def test_geometry_of_presets():
    """Pillar solid fraction and electrode placement of the workloads (Results, Fig. 1 text)."""
    c3 = make_case("c3")
    x, y, z = c3.coords()
    pil = (c3.flags == GROUND) & (z >= 1) & (z <= 10)
    assert pil.sum() == (c3.n[0] // 12 * 6 + min(6, c3.n[0] % 12)) * (c3.n[1] // 12 * 6 + min(6, c3.n[1] % 12)) * 10
    e = c3.flags == ELECTRODE0
    assert set(np.unique(x[e])) == set(range(134, 198)) and set(np.unique(z[e])) == {95}
    c2 = make_case("c2")
    x, y, z = c2.coords()
    e = c2.flags == ELECTRODE0
    assert set(np.unique(x[e])) == set(range(208, 272)) and set(np.unique(y[e])) == {255}
    assert abs(c2.phi[:, c2.flags == FLUID].sum(0) - 1).max() < 1e-12


def test_zero_rates_and_densities_mean_the_defaults(L):
    """A zero-initialised s_high or rho (a C caller's zeroed struct) is the default 1."""
    case = make_case("c2s")
    _ctx(case, s_high=0.0, rho=(0.0, 0.0, 0.0))
    _ctx(case, s_high=1.7, rho=(1.0, 0.0, 1.0))
    _ctx(case, rho=(998.0, 970.0, 1.2))          # the paper's Table 1 densities are accepted
    _ctx(case, gamma12=1e-3, gamma13=2.5e-3, gamma23=1e-3)   # cloaking: Upsilon_2 < 0


@pytest.mark.parametrize("name", ["c1", "c1s", "c2", "c2s", "c3", "c3s", "c4", "c4s", "c5"])
def test_preset_matches_the_input_generator(L, name):
    """ehdlb_preset (host-only, no device) builds the same lattice, parameters, node flags
    and initial phase fields as the seeded input generator the tests use: flags and
    parameters bit for bit; the phase fields are sums and products of interface profiles
    0.5 (1 + tanh(.)) in [0, 1], and numpy's vectorised tanh and the C library's differ by one
    unit in the last place on about a quarter of the arguments, so they agree to within the
    three units of 1.0 (6.7e-16) that such a difference can become through Phi_3 = 1 - Phi_1 -
    Phi_2, and exactly wherever the two tanh agree."""
    from paper_2608_12868_amd.sim import preset
    seed = 7 if name in ("c1", "c1s") else 0
    lat, p, flags, phi = preset(name, seed)
    case = make_case(name, seed=seed)
    assert lat.dim == case.dim and tuple(lat.n) == case.n and tuple(lat.periodic) == case.periodic
    assert lat.precision == (L.FP64 if case.precision == "fp64" else L.FP32_DEV)
    assert np.array_equal(flags, case.flags)
    ref = case.params
    for k in ("tau_flow", "eps", "cond", "body_force", "rho"):
        assert list(getattr(p, k)) == list(ref[k]), k
    assert list(p.electrode_volts) == list(ref["electrode_volts"])
    for k in ("mobility", "width", "gamma12", "gamma13", "gamma23", "cos12", "cos13", "cos23",
              "charge_diffusion", "poisson_tol", "s_high"):
        assert getattr(p, k) == ref[k], k
    assert p.ehd == ref["ehd"] and p.poisson_max_iter == ref["poisson_max_iter"]
    assert p.poisson_check_every == ref["poisson_check_every"]
    diff = np.abs(phi - case.phi).max()
    same = float(np.mean(phi == case.phi))
    print(name, "max difference", diff, "bit-identical fraction", same)
    assert diff <= 3 * 2.0 ** -52
    assert np.all(phi[:, case.flags != FLUID] == 0.0)


def test_preset_rejects_unknown_ids(L):
    lat, p = L.Lattice(), L.Params()
    assert L.lib().ehdlb_preset(99, C.byref(lat), C.byref(p), None, None, 0) == L.EINVAL


def test_bandwidth_probe_rejects_bad_arguments(L):
    """Every rejection happens before anything is queued, so no device is needed."""
    lib = L.lib()
    fake = C.c_void_p(4096)
    dims = (C.c_int32 * 3)(8, 6, 5)
    assert lib.ehdlb_bandwidth_probe(4, fake, fake, 64, None, 0, 0, None) == L.EINVAL     # unknown kind
    assert lib.ehdlb_bandwidth_probe(0, None, fake, 64, None, 0, 0, None) == L.EINVAL     # NULL source
    assert lib.ehdlb_bandwidth_probe(0, fake, fake, 40, None, 0, 0, None) == L.EINVAL     # not 16-byte sized
    assert lib.ehdlb_bandwidth_probe(0, C.c_void_p(4100), fake, 64, None, 0, 0, None) == L.EINVAL  # misaligned
    assert lib.ehdlb_bandwidth_probe(1, fake, fake, 6, None, 0, 0, None) == L.EINVAL      # not 4-byte sized
    need = 2 * 19 * 8 * 6 * 5 * 4
    assert lib.ehdlb_bandwidth_probe(2, fake, fake, need, None, 19, 2, None) == L.EINVAL  # no dims
    assert lib.ehdlb_bandwidth_probe(2, fake, fake, need - 4, dims, 19, 2, None) == L.EINVAL  # too small
    assert lib.ehdlb_bandwidth_probe(2, fake, fake, need, dims, 9, 2, None) == L.EINVAL   # D2Q9 with nz > 1
    assert lib.ehdlb_bandwidth_probe(3, fake, fake, need, dims, 15, 2, None) == L.EINVAL  # unknown velocity set
    assert lib.ehdlb_bandwidth_probe(2, fake, fake, need * 4, dims, 19, 6, None) == L.EINVAL  # too many families
