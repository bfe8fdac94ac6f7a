"""lqcd_apply_native_noalloc (no device allocation; the library's static
scratch array) against lqcd_apply_native on the same inputs: two calls in a
row on lattices of decreasing size, every precision, results identical (the
same kernels and launch shapes), and the size limit reported as EINVAL."""

import numpy as np
import pytest

import fieldgen as fg
from paper_2303_05883_amd import lqcd
from tests.gpuutil import lattice, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def schur_both(lat, prec, src):
    torch = torch_cuda()
    nb = lat.field_bytes(prec)
    inp = torch.empty(nb, dtype=torch.uint8, device="cuda")
    lat.import_field(prec, 0, src, inp)
    o_alloc = torch.empty(nb, dtype=torch.uint8, device="cuda")
    o_none = torch.empty(nb, dtype=torch.uint8, device="cuda")
    lat.apply_native("DPREC_SCHUR", prec, inp, o_alloc)
    lat.apply_native_noalloc("DPREC_SCHUR", prec, inp, o_none)
    a = torch.zeros_like(src)
    b = torch.zeros_like(src)
    lat.export_field(prec, 0, o_alloc, a)
    lat.export_field(prec, 0, o_none, b)
    torch.cuda.synchronize()
    return a, b


def test_noalloc_schur_matches_allocating_entry_point():
    torch = torch_cuda()
    for dims, seed in (((8, 8, 8, 16), 71), ((4, 4, 4, 8), 72)):  # second call: smaller input
        U = fg.gauge_field(dims, seed, "smooth", 0.3)
        src = to_dev(fg.gaussian_spinor(dims, seed + 1))
        lat = lattice(dims, U, 0.137, 1.0)
        for prec in (lqcd.F64, lqcd.F32, lqcd.F16):
            a, b = schur_both(lat, prec, src)
            assert torch.count_nonzero(a) > 0
            assert torch.equal(a, b), (dims, prec)
        # operators without scratch go through unchanged
        nb = lat.field_bytes(lqcd.F64)
        inp = torch.empty(nb, dtype=torch.uint8, device="cuda")
        lat.import_field(lqcd.F64, 1, src, inp)
        o1 = torch.zeros(nb, dtype=torch.uint8, device="cuda")
        o2 = torch.zeros(nb, dtype=torch.uint8, device="cuda")
        lat.apply_native("HOP_EO", lqcd.F64, inp, o1)
        lat.apply_native_noalloc("HOP_EO", lqcd.F64, inp, o2)
        torch.cuda.synchronize()
        assert torch.equal(o1, o2)
        lat.close()


def test_noalloc_rejects_fields_beyond_the_scratch():
    torch = torch_cuda()
    dims = (32, 32, 32, 48)  # FP64 half field 151 MB > 128 MiB
    lat = lqcd.Lattice(dims, -1)
    nb = lat.field_bytes(lqcd.F64)
    buf = torch.empty(2 * nb, dtype=torch.uint8, device="cuda")
    with pytest.raises(lqcd.LqcdError) as e:
        lat.apply_native_noalloc("DPREC_SCHUR", lqcd.F64, buf[:nb], buf[nb:])
    assert e.value.status == lqcd.EINVAL
    lat.close()
