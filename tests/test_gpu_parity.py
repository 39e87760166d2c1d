"""GPU parity: every degree p = 1..7 and every precision path of libfem against the FP64 oracle,
element by element, on seeded jittered meshes that span several work items with ragged tails.
Calls go through the C ABI (paper_1310_1191_amd.fem)."""
import numpy as np
import pytest

from gpu_cases import TOL_A, TOL_B, log, oracle_uniform, rel_fro, rel_vec, to_dev

pytestmark = pytest.mark.gpu

PRECS = ["fp64", "fp32", "split_bf16", "split_fp16", "bf16"]


@pytest.fixture(scope="module")
def fem():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1310_1191_amd import fem as F
    F.fem_init(0)
    return F


@pytest.mark.parametrize("p", range(1, 8))
@pytest.mark.parametrize("prec", PRECS)
def test_uniform_parity(fem, p, prec):
    import torch
    geom, coef, A_ref, b_ref, fl = oracle_uniform(p)
    g, c = to_dev(geom, coef)
    status = torch.zeros(2, dtype=torch.int32, device="cuda")
    A, b = fem.integrate(g, c, p, precision=prec, status=status)
    torch.cuda.synchronize()
    A = A.double().cpu().numpy()
    b = b.double().cpu().numpy()
    ea = rel_fro(A, A_ref)
    eb = rel_vec(b, b_ref)
    log(f"[parity] p={p} prec={prec} nel={geom.shape[0]} errA max={ea.max():.3e} "
        f"p99={np.percentile(ea, 99):.3e} med={np.median(ea):.3e} errb max={eb.max():.3e}")
    assert status.cpu().tolist() == [0, 0]
    assert np.isfinite(A).all()
    assert ea.max() <= TOL_A[prec], f"max rel Frobenius error {ea.max():.3e}"
    assert eb.max() <= TOL_B[prec], f"max rel load-vector error {eb.max():.3e}"


@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_fp16"])
def test_p1_poisson_workload(fem, prec):
    import torch
    geom, coef, A_ref, b_ref, _ = oracle_uniform(1, "poisson")
    g, c = to_dev(geom, coef)
    A, b = fem.integrate(g, c, 1, precision=prec)
    torch.cuda.synchronize()
    ea = rel_fro(A.double().cpu().numpy(), A_ref)
    log(f"[parity] poisson p=1 prec={prec} nel={geom.shape[0]} errA max={ea.max():.3e}")
    assert ea.max() <= TOL_A[prec]
    # row sums of the pure-diffusion matrix vanish
    rs = np.abs(A.double().cpu().numpy().sum(axis=2)).max()
    assert rs <= 10 * TOL_A[prec] * np.abs(A_ref).max()


def test_zero_elements_is_a_no_op(fem):
    import torch
    g = torch.zeros((0, 8, 3), dtype=torch.float64, device="cuda")
    c = torch.zeros((0, 14), dtype=torch.float64, device="cuda")
    A, b = fem.integrate(g, c, 3, precision="fp32")
    torch.cuda.synchronize()
    assert A.shape == (0, 64, 64)


@pytest.mark.parametrize("prec", ["fp64", "split_fp16"])
def test_single_element_each_degree(fem, prec):
    import torch
    for p in range(1, 8):
        geom, coef, A_ref, b_ref, _ = oracle_uniform(p)
        g, c = to_dev(geom[:1], coef[:1])
        A, b = fem.integrate(g, c, p, precision=prec)
        torch.cuda.synchronize()
        ea = rel_fro(A.double().cpu().numpy(), A_ref[:1])
        assert ea.max() <= TOL_A[prec], (p, ea.max())


def test_bad_arguments_return_codes(fem):
    import torch
    g, c = to_dev(*oracle_uniform(2)[:2])
    A = torch.empty((g.shape[0], 27, 27), dtype=torch.float32, device="cuda")
    co = fem.make_coeffs("fp32", fem.ELEMENT, c)
    assert fem.fem_integrate(g.shape[0], 8, g.data_ptr(), co, A.data_ptr(), None, None) == fem.FEM_EDEGREE
    assert fem.fem_integrate(-1, 2, g.data_ptr(), co, A.data_ptr(), None, None) == fem.FEM_EINVAL
    assert fem.fem_integrate(g.shape[0], 2, None, co, A.data_ptr(), None, None) == fem.FEM_EINVAL
    assert fem.fem_integrate(g.shape[0], 0, g.data_ptr(), co, A.data_ptr(), None, None) == fem.FEM_EDEGREE
    co.precision = 9
    assert fem.fem_integrate(g.shape[0], 2, g.data_ptr(), co, A.data_ptr(), None, None) == fem.FEM_EINVAL
    co = fem.make_coeffs("fp32", fem.FIELD, c)
    assert fem.fem_integrate(g.shape[0], 2, g.data_ptr(), co, A.data_ptr(), None, None) == fem.FEM_EINVAL


def test_status_counts_inverted_and_nonfinite(fem):
    import oracle
    import torch
    geom, coef = oracle_uniform(2)[:2]
    geom = geom[:8].copy()
    coef = coef[:8].copy()
    geom[3] = geom[3][[1, 0, 3, 2, 5, 4, 7, 6]]   # mirrored: detJ < 0
    geom[5, 2, 1] = np.nan
    A_ref, b_ref, fl = oracle.integrate(geom, coef, p=2)
    # a NaN coordinate makes detJ NaN: "not > 0" and non-finite, on both sides
    assert fl.tolist() == [0, 0, 0, 1, 0, 3, 0, 0]
    g, c = to_dev(geom, coef)
    status = torch.zeros(2, dtype=torch.int32, device="cuda")
    for prec in ["fp64", "split_fp16"]:
        status.zero_()
        A, b = fem.integrate(g, c, 2, precision=prec, status=status)
        torch.cuda.synchronize()
        assert status.cpu().tolist() == [2, 1]
        ok = [0, 1, 2, 3, 4, 6, 7]   # the inverted element is integrated with the signed detJ
        ea = rel_fro(A.double().cpu().numpy()[ok], A_ref[ok])
        assert ea.max() <= TOL_A[prec]
        assert not np.isfinite(A[5].cpu().numpy()).all()


def test_deterministic_bitwise(fem):
    import torch
    g, c = to_dev(*oracle_uniform(4)[:2])
    A1, b1 = fem.integrate(g, c, 4, precision="split_bf16")
    A2, b2 = fem.integrate(g, c, 4, precision="split_bf16")
    torch.cuda.synchronize()
    assert torch.equal(A1, A2) and torch.equal(b1, b2)
