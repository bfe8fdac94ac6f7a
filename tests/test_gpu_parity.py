"""Parity of every operator the library applies against the CPU oracle.

Each case builds the same seeded fields on the host, applies the operator
through the C ABI on the GPU and with the oracle, and compares element by
element (rel-L2): <= 1e-13 in FP64, <= 1e-5 in FP32, <= 5e-3 in FP16.
Lattices span several workgroups and ragged tails (4^4 = 128 sites per
parity; 4x6x8x10 = 960; 8^3x16 = 4096; 2x2x2x4 has coinciding forward and
backward neighbours).
"""

import numpy as np
import pytest

import fieldgen as fg
from oracle import dirac
from tests.gpuutil import TOL, from_dev, lattice, to_dev

pytestmark = pytest.mark.gpu

DIMS = [(4, 4, 4, 4), (2, 2, 2, 4), (4, 6, 8, 10), (8, 8, 8, 16)]


def oracle_op(op: dirac.Operator, name: str, psi):
    m = dirac.mask
    return {
        "D": lambda: op.D(psi),
        "DEE": lambda: op.Dee(psi),
        "DOO": lambda: op.Doo(psi),
        "DEO": lambda: op.Deo(psi),
        "DOE": lambda: op.Doe(psi),
        "HOP_EO": lambda: m(op.hop(m(psi, 1)), 0),
        "HOP_OE": lambda: m(op.hop(m(psi, 0)), 1),
        "DPREC_SCHUR": lambda: op.schur(m(psi, 0)),
        "DPREC_PAPER": lambda: op.dprec(m(psi, 0)),
        "DEE_INV": lambda: op.site_inverse(0, psi),
        "DOO_INV": lambda: op.site_inverse(1, psi),
    }[name]()


CASES = {}


def case(dims, csw, t_bc):
    key = (dims, csw, t_bc)
    if key not in CASES:
        U = fg.gauge_field(dims, 7, "smooth", 0.4)
        psi = fg.gaussian_spinor(dims, 8)
        op = dirac.Operator(U, 0.1285, csw, t_bc)
        lat = lattice(dims, U, 0.1285, csw, t_bc)
        CASES[key] = (U, psi, op, lat)
    return CASES[key]


OPNAMES = ["D", "DEE", "DOO", "DEO", "DOE", "HOP_EO", "HOP_OE", "DPREC_SCHUR", "DPREC_PAPER", "DEE_INV", "DOO_INV"]


# hop launch shapes: (block, lanes per site, block-to-XCD mapping, non-temporal links)
SHAPES = [(256, 1, 1, 0), (64, 4, 1, 1), (192, 4, 0, 0), (128, 1, 0, 1), (128, 1, 2, 1), (256, 4, 2, 0),
          (128, 2, 1, 1), (256, 2, 0, 0), (64, 2, 2, 1)]


def march_shapes(dims):
    """Plane-march shapes (lanes = Lx/2 x rows, split 0, z planes per block, nt)
    that are valid on dims: whole-plane tiles and half-plane tiles with halo rows."""
    lxh, ly, lz = dims[0] // 2, dims[1], dims[2]
    out = []
    for rows in (ly, ly // 2):
        if rows < 2 or ly % rows or lxh * rows > 512:
            continue
        for zc in (1, 2, 4):
            if lz % zc == 0 and lxh * rows * zc >= 16:
                out.append((lxh * rows, 0, zc, 1))
                break
    return out


def shapes_for(dims):
    return [s for s in SHAPES if s[2] != 2 or dims[2] % 8 == 0] + march_shapes(dims)
REFS = {}


def oracle_ref(key, op, name, psi):
    k = key + (name,)
    if k not in REFS:
        REFS[k] = oracle_op(op, name, psi)
    return REFS[k]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("csw", [0.0, 1.0])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_apply_matches_oracle(dims, csw, prec):
    U, psi, op, lat = case(dims, csw, -1)
    x = to_dev(psi)
    out = to_dev(np.zeros_like(psi))
    bad = {}
    for shape in shapes_for(dims):
        lat.set_hop_shape(prec, *shape)
        for name in OPNAMES:
            lat.apply(name, prec, x, out)
            err = dirac.rel_l2(from_dev(out), oracle_ref((dims, csw), op, name, psi))
            if not err <= TOL[prec]:
                bad[(shape, name)] = err
    lat.set_hop_shape(prec)
    assert not bad, f"{dims} csw={csw} prec={prec}: {bad}"


def test_launch_shapes_agree_in_fp64():
    """The FP64 operator does not depend on the launch shape beyond the order in
    which the eight hops of a site are added."""
    U, psi, op, lat = case((4, 6, 8, 10), 1.0, -1)
    x = to_dev(psi)
    outs = []
    for shape in shapes_for((4, 6, 8, 10)):
        lat.set_hop_shape(0, *shape)
        out = to_dev(np.zeros_like(psi))
        lat.apply("DPREC_SCHUR", 0, x, out)
        outs.append(from_dev(out))
    lat.set_hop_shape(0)
    for o in outs[1:]:
        assert np.abs(o - outs[0]).max() <= 1e-14 * np.abs(outs[0]).max()


def test_periodic_time_boundary():
    U, psi, op, lat = case((4, 4, 4, 6), 1.0, +1)
    out = to_dev(np.zeros_like(psi))
    lat.apply("D", 0, to_dev(psi), out)
    assert dirac.rel_l2(from_dev(out), op.D(psi)) <= 1e-13


def test_host_pointers_match_device_pointers():
    U, psi, op, lat = case((4, 6, 8, 10), 1.0, -1)
    host_out = np.zeros_like(psi)
    lat.apply("DPREC_SCHUR", 0, psi, host_out)
    dev_out = to_dev(np.zeros_like(psi))
    lat.apply("DPREC_SCHUR", 0, to_dev(psi), dev_out)
    assert np.array_equal(host_out, from_dev(dev_out))


def test_parity_blocks_sum_to_full_operator():
    U, psi, op, lat = case((4, 6, 8, 10), 1.0, -1)
    total = np.zeros_like(psi)
    for name in ["DEE", "DEO", "DOE", "DOO"]:
        out = np.zeros_like(psi)
        lat.apply(name, 0, psi, out)
        total += out
    full = np.zeros_like(psi)
    lat.apply("D", 0, psi, full)
    assert np.abs(total - full).max() <= 1e-14 * np.abs(full).max()


def test_fp16_zero_sites_and_point_source():
    dims = (4, 4, 4, 4)
    U, psi, op, lat = case(dims, 1.0, -1)
    src = fg.point_source(dims, 2, 1)
    out = to_dev(np.zeros_like(src))
    for prec in (0, 1, 2):
        lat.apply("D", prec, to_dev(src), out)
        assert dirac.rel_l2(from_dev(out), op.D(src)) <= TOL[prec]
    zero = np.zeros_like(src)
    lat.apply("D", 2, to_dev(zero), out)
    assert not np.any(from_dev(out))


def test_gamma5_hermiticity_on_gpu():
    U, psi, op, lat = case((4, 6, 8, 10), 1.0, -1)
    phi = fg.gaussian_spinor((4, 6, 8, 10), 99)
    a = np.zeros_like(psi)
    lat.apply("D", 0, psi, a)
    b = np.zeros_like(psi)
    lat.apply("D", 0, dirac.gamma5(phi), b)
    lhs = np.vdot(phi, a)
    rhs = np.vdot(dirac.gamma5(b), psi)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_rejects_non_su3_and_nan():
    from paper_2303_05883_amd import lqcd
    dims = (4, 4, 4, 4)
    U = fg.gauge_field(dims, 1, "haar").copy()
    lat = lqcd.Lattice(dims, -1)
    bad = U.copy()
    bad[1, 2, 3, 0, 2] *= 1.001
    with pytest.raises(lqcd.LqcdError) as e:
        lat.set_gauge(to_dev(bad))
    assert e.value.status == lqcd.ENOTSU3
    bad = U.copy()
    bad[0, 0, 0, 1, 3, 1, 1] = np.nan
    with pytest.raises(lqcd.LqcdError) as e:
        lat.set_gauge(to_dev(bad))
    assert e.value.status == lqcd.EINVAL
    with pytest.raises(lqcd.LqcdError) as e:
        lat.apply("D", 0, np.zeros((4, 4, 4, 4, 4, 3), complex), np.zeros((4, 4, 4, 4, 4, 3), complex))
    assert e.value.status == lqcd.ESTATE
    lat.set_gauge(to_dev(U))
    lat.set_clover(0.12, 1.0)
    psi = fg.gaussian_spinor(dims, 2)
    psi[0, 0, 0, 0, 0, 0] = np.inf
    with pytest.raises(lqcd.LqcdError) as e:
        lat.solve(psi, np.zeros_like(psi))
    assert e.value.status == lqcd.EINVAL
