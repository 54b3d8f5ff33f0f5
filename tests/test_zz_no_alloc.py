"""The allocation-free residual (lskum_residual_noalloc) against the state
residual (lskum_residual) through the C ABI: the same kernels on the same
input, so the residual field and its norm must agree bit for bit.  Two calls
in a row, the second on a smaller cloud (the shared scratch array keeps the
first call's contents), and a cloud beyond the scratch array's capacity is
refused.
"""
import numpy as np
import pytest

from paper_2406_07441_amd import cloudgen as cg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lk():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_07441_amd import lskum
    lskum.lib()
    return lskum


def state_after(lk, gc, mach, aoa, prm, steps):
    st = lk.State(gc, mach, aoa, prm)
    for _ in range(steps):
        st.step()
    U = st.get_U()
    st.set_U(U)
    R, res = st.residual()
    st.close()
    return U, R, res


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_residual_equals_state_residual(lk, order):
    import torch
    cases = [
        # 6,400 points, limiter on, 5 iterations into the lifting case
        (cg.cloud_6400(), 0.63, 2.0, dict(cfl=100.0, inner_iters=1, limiter=1, limiter_k=5.0), 5),
        # then a smaller cloud with two inner iterations and the kinetic far field
        (cg.ogrid(64, 16, r=1.15), 0.5, 3.0,
         dict(cfl=50.0, inner_iters=2, farfield=lk.FARFIELD_KINETIC), 3),
    ]
    for cloud, mach, aoa, kw, steps in cases:
        gc = lk.Cloud(cloud)
        prm = lk.default_params(**kw)
        U, R_ref, res_ref = state_after(lk, gc, mach, aoa, prm, steps)
        Ud = torch.tensor(U, dtype=torch.float64, device="cuda")
        Rd = torch.full_like(Ud, float("nan"))
        rd = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        lk.residual_noalloc(gc, mach, aoa, prm, Ud, Rd, rd)
        torch.cuda.synchronize()
        R = Rd.cpu().numpy()
        res, bad = rd.cpu().numpy()
        print(f"n={cloud.n}: res {res:.12e} / {res_ref:.12e}, max |dR| {np.abs(R - R_ref).max():.3e}")
        assert np.array_equal(R, R_ref)
        assert res == res_ref and bad == 0.0
        # the norm alone (R = NULL)
        rd2 = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        lk.residual_noalloc(gc, mach, aoa, prm, Ud, None, rd2)
        torch.cuda.synchronize()
        assert rd2[0].item() == res_ref
        gc.close()


def test_noalloc_residual_flags_a_nonphysical_state(lk):
    import torch
    cloud = cg.ogrid(64, 16, r=1.15)
    gc = lk.Cloud(cloud)
    prm = lk.default_params()
    st = lk.State(gc, 0.5, 0.0, prm)
    U = st.get_U()
    st.close()
    U[0, 100] = -1.0   # negative density at one interior point
    Ud = torch.tensor(U, dtype=torch.float64, device="cuda")
    rd = torch.zeros(2, dtype=torch.float64, device="cuda")
    lk.residual_noalloc(gc, 0.5, 0.0, prm, Ud, None, rd)
    torch.cuda.synchronize()
    assert rd[1].item() == 1.0
    gc.close()


def test_noalloc_residual_refuses_a_cloud_beyond_the_scratch(lk):
    import torch
    cap = lk.residual_noalloc_max_points()
    assert 163840 <= cap < 200000
    cloud = cg.ogrid(640, 300)   # 192,000 points
    assert cloud.n > cap
    gc = lk.Cloud(cloud)
    U = torch.zeros((4, cloud.n), dtype=torch.float64, device="cuda")
    rd = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(lk.LskumError) as e:
        lk.residual_noalloc(gc, 0.5, 0.0, lk.default_params(), U, None, rd)
    assert e.value.code == lk.ERR_ARG
    gc.close()
