"""The allocation-free product mtf_matvec_noalloc (static device scratch) against mtf_matvec.

Same kernels, same summation order: the results must agree bit for bit.  Two calls in a row on
one GPU, the second on a smaller problem (the scratch keeps the first call's contents), and a
problem too large for the scratch is rejected before any device work.  Runs last (its file name
sorts after every other test file).
"""
import numpy as np
import pytest

import mtf_inputs as mi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2502_10907_amd as mtf  # noqa: E402


def _problem(cfg, precisions):
    m = cfg["mesh"]
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
    for pr in precisions:
        P.assemble(pr)
    return P


def _vectors(P, nrhs, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn((nrhs, P.N), dtype=torch.complex128, generator=g).to("cuda")
    return x, torch.zeros_like(x), torch.full_like(x, complex(np.nan, np.nan))


def test_noalloc_product_equals_matvec_on_two_calls():
    big = _problem(mi.config_cube(2, 8), (mtf.FP64, mtf.FP32_MIXED))        # N = 6,912
    small = _problem(mi.config_sphere(1), (mtf.FP64, mtf.FP32_MIXED))       # N = 480
    print(f"\n[case] no-alloc product: cube 2x2x2 h=1/8 (N={big.N}) then sphere (N={small.N})", flush=True)
    assert small.N < big.N
    for P, nrhs, seed in ((big, 2, 0), (small, 1, 1)):
        for prec in (mtf.FP64, mtf.FP32_MIXED):
            x, y_ref, y = _vectors(P, nrhs, seed)
            P.matvec(x, y_ref, prec)
            P.matvec_noalloc(x, y, prec)
            torch.cuda.synchronize()
            a, b = y_ref.cpu().numpy(), y.cpu().numpy()
            assert np.all(np.isfinite(b))
            assert np.array_equal(a, b), (P.N, prec, np.abs(a - b).max())
    # the larger problem again after the smaller one
    x, y_ref, y = _vectors(big, 1, 2)
    big.matvec(x, y_ref, mtf.FP64)
    big.matvec_noalloc(x, y, mtf.FP64)
    torch.cuda.synchronize()
    assert np.array_equal(y_ref.cpu().numpy(), y.cpu().numpy())


def test_noalloc_rejects_what_the_scratch_cannot_hold():
    cfg = mi.config_cube(4, 24)                  # N = 103,680: about 69 MB of partial sums
    m = cfg["mesh"]
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
    x = torch.zeros((1, P.N), dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(mtf.MTFError) as e:
        P.matvec_noalloc(x, y, mtf.FP64)
    assert e.value.code == -1 and "scratch" in str(e.value)
    with pytest.raises(mtf.MTFError):
        P.matvec_noalloc(x, y, mtf.BF16_SPLIT)
