"""The V-cycle entry point that allocates nothing (mgpcg_mg_vcycle_noalloc).

Through the C ABI: its results equal mgpcg_mg_vcycle's bit for bit, on two
calls in a row on different problems, the second smaller; it leaves the
device's free memory unchanged where the allocating entry point's first call
does not; and it rejects a natural-layout problem above its staging limit.
"""
import numpy as np
import pytest

from paper_2304_08232_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_08232_amd import mgpcg
    mgpcg.lib()
    return mgpcg


def dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


CASES = [  # (dims, kwargs): the second of each pair is smaller than the first
    ((64, 64, 64), {}), ((16, 16, 16), {}),
    ((32, 32, 32), {"colour_order": 1}), ((16, 8, 8), {"colour_order": 1}),
    ((32, 32, 32), {"mg_dtype": "fp32"}), ((16, 16, 16), {"mg_dtype": "fp32"}),
    ((32, 16, 16), {"nrhs": 4}), ((16, 16, 16), {"nrhs": 2}),
    ((16, 16, 16), {"smoother": "sequential"}), ((8, 8, 8), {"smoother": "sequential"}),
]


@pytest.mark.parametrize("first", range(0, len(CASES), 2))
def test_noalloc_equals_vcycle_twice(mg, first):
    for dims, kw in CASES[first:first + 2]:
        print(f"noalloc {dims} {kw}", flush=True)
        p = mg.Problem(dims, levels=3 if dims == (8, 8, 8) else 4, **kw)
        n = p.n(0) * p.nrhs
        r = dev(inputs.uniform(33, n))
        for layout in (mg.NATURAL, mg.INTERNAL):
            ri = r if layout == mg.NATURAL else p.to_internal(r)
            z_ref = torch.zeros_like(ri)
            z_new = torch.full_like(ri, np.nan)
            mg.mgpcg_mg_vcycle(p.h, ri, z_ref, layout)
            mg.mgpcg_mg_vcycle_noalloc(p.h, ri, z_new, layout)
            torch.cuda.synchronize()
            assert torch.equal(z_new, z_ref), (dims, kw, layout)
        p.close()


def test_noalloc_allocates_nothing(mg):
    p = mg.Problem((64, 64, 64), levels=4)
    r = dev(inputs.uniform(34, 64 ** 3))
    z = torch.zeros_like(r)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        mg.mgpcg_mg_vcycle_noalloc(p.h, r, z, mg.NATURAL)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    # the allocating entry point's first call takes its staging buffers (6 MB here)
    mg.mgpcg_mg_vcycle(p.h, r, z, mg.NATURAL)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] < free0
    p.close()


def test_noalloc_rejects_above_limit(mg):
    p = mg.Problem((136, 128, 128), levels=4)  # 2,228,224 values > 2^21
    r = torch.zeros(p.n(0), dtype=torch.float64, device="cuda")
    z = torch.zeros_like(r)
    with pytest.raises(mg.MGPCGError, match="staging limit"):
        mg.mgpcg_mg_vcycle_noalloc(p.h, r, z, mg.NATURAL)
    # internal layout stages nothing and has no limit
    ri = p.to_internal(dev(inputs.uniform(35, p.n(0))))
    z_ref, z_new = torch.zeros_like(ri), torch.zeros_like(ri)
    mg.mgpcg_mg_vcycle(p.h, ri, z_ref, mg.INTERNAL)
    mg.mgpcg_mg_vcycle_noalloc(p.h, ri, z_new, mg.INTERNAL)
    torch.cuda.synchronize()
    assert torch.equal(z_new, z_ref)
    p.close()
