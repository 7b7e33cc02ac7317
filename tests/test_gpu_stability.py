"""High-order stability of the radial tables (Sec. 3.1, Fig. 1) on the GPU.

Orthogonality on Gauss-Legendre rings, E(n) = max over m and n' of
|2(n+1) sum_r w_r R_nm R_n'm - delta_nn'|, for the FP64 eq. (7) table and
for the number formats the projection operand holds it in.  Each operand
entry carries a relative error of at most u (FP32: 2^-24; hi + lo bfloat16:
2^-16 + 2^-24; hi + lo half: 2^-22), and by the Cauchy-Schwarz
inequality with 2(n+1) sum_r w_r R_nm^2 = 1 the products then move E(n) by
at most 2u(1 + u) beyond the FP64 table's own E(n).  The host rule that forms
the split values for orders the moment kernels do not serve is first checked
bit for bit against the operand the library builds on the device.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

U = {"f32": 2.0 ** -24, "bf16x2": 2.0 ** -16 + 2.0 ** -24, "f16x2": 2.0 ** -22}


@pytest.fixture(scope="module")
def zm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2304_14492_amd as m
    return m


@pytest.mark.parametrize("dtype,neumann", [("f32", False), ("bf16x2", True), ("f16x2", False), ("f16x2", True)])
def test_host_split_rule_equals_device_operand(zm, dtype, neumann):
    from paper_2304_14492_amd import stability
    plan = zm.Plan(255, 1024, 1024, dtype=dtype, neumann=neumann, rings=257, angles=1024, rule="gauss_legendre")
    dev = stability.operand_effective(plan)
    host = stability.split_effective(plan.radial_table(), stability.fold_factors(plan), dtype)
    assert np.array_equal(dev, host)


def test_orthogonality_to_order_500(zm):
    from paper_2304_14492_amd import stability
    plan = zm.Plan(500, 2048, 2048, dtype="f32", rings=502, angles=1024, rule="gauss_legendre")
    res = stability.sweep(plan)
    for row in res["bands"]:
        print("n %3d-%3d  " % tuple(row["n"]) + "  ".join(f"{k} {row[k]:.2e}" for k in ("f64", "f32", "bf16x2", "f16x2")))
    E64 = res["curves"]["f64"]
    assert E64.max() <= 1e-10
    for fmt, u in U.items():
        bound = 2 * u * (1 + u) + E64 + 1e-12
        assert np.all(res["curves"][fmt] <= bound), (fmt, float(np.max(res["curves"][fmt] / bound)))
