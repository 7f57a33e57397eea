"""The allocation-free right-hand side ns_rhs_static (static device scratch,
for callers that cannot allocate) against ns_rhs of a solver, through the C
ABI: two calls in a row, the second on a smaller problem, in both
precisions, 3D and 2D Boussinesq; sizes beyond the scratch are refused."""
import numpy as np
import pytest

from gpu_util import announce, per_field_rel_l2
from paper_1810_10197_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ns():
    from paper_1810_10197_amd import ns as mod
    return mod


def static_rhs(ns, torch, cfg, nus, u):
    x = torch.from_numpy(np.ascontiguousarray(u)).to("cuda")
    f = torch.full_like(x, complex(np.nan, np.nan))    # every entry must be written
    st = torch.cuda.current_stream()
    ns.ns_rhs_static(cfg, nus, x.data_ptr(), f.data_ptr(), st.cuda_stream)
    st.synchronize()
    return f.cpu().numpy()


CASES = [
    # (dim, n, batch, precision, scalar): the first case larger than the second
    ((3, 64, 2, "fp32", 0), (3, 32, 1, "fp32", 0)),
    ((3, 64, 1, "fp64", 0), (3, 16, 3, "fp64", 0)),
    ((2, 1024, 1, "fp32", 1), (2, 256, 2, "fp32", 1)),
]


@pytest.mark.parametrize("first,second", CASES)
def test_static_rhs_equals_solver_rhs(ns, first, second):
    import torch
    for dim, n, batch, prec, scalar in (first, second):
        announce("ns_rhs_static dim=%d n=%d B=%d %s" % (dim, n, batch, prec))
        if dim == 3:
            fields = np.stack([inputs.random_isotropic(n, 40 + m, k0=n / 8.0) for m in range(batch)])
            kw = {}
        else:
            fields = np.stack([inputs.rayleigh_taylor2d(n) for _ in range(batch)])
            fields[:, :2] = np.stack([inputs.tgv2d(n) * (m + 1) for m in range(batch)])
            kw = {"scalar": 1, "ri": 0.5, "kappa": 1e-4}
        nus = 10.0 ** (-3.0 + 0.3 * np.arange(batch))
        s = ns.Solver(dim=dim, n=n, batch=batch, nu=nus, rhs_precision=prec, **kw)
        ref = s.rhs(fields).cpu().numpy()
        cfg = s.cfg
        s.close()
        assert 0 < ns.ns_rhs_static_bytes(cfg) <= ns.NS_STATIC_SCRATCH_BYTES
        got = static_rhs(ns, torch, cfg, nus, fields)
        assert np.all(np.isfinite(got.view(np.float64)))
        for m in range(batch):
            if prec == "fp64":
                err = np.abs(got[m] - ref[m]).max() / np.abs(ref[m]).max()
                assert err <= 1e-12, (m, err)
            else:
                errs = per_field_rel_l2(got[m], ref[m])
                assert max(errs) <= 1e-6, (m, errs)


def test_sizes_beyond_the_scratch_are_refused(ns):
    import torch
    cfg = ns.NsConfig(3, 128, 1, ns.NS_FP32, 0, 0.0, 0.0, 0.0, 0.0, 0)
    assert ns.ns_rhs_static_bytes(cfg) > ns.NS_STATIC_SCRATCH_BYTES
    x = torch.zeros((1, 3, 128, 128, 65), dtype=torch.complex128, device="cuda")
    f = torch.zeros_like(x)
    with pytest.raises(ns.NsError) as e:
        ns.ns_rhs_static(cfg, np.array([0.01]), x.data_ptr(), f.data_ptr(),
                         torch.cuda.current_stream().cuda_stream)
    assert e.value.status == ns.NS_ERR_SCRATCH
    big = ns.NsConfig(3, 16, ns.NS_STATIC_MAX_BATCH + 1, ns.NS_FP32, 0, 0.0, 0.0, 0.0, 0.0, 0)
    assert ns.ns_rhs_static_bytes(big) == 0
