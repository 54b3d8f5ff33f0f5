"""Parity at the benchmark sizes, in the launch configuration the benchmark times.

* 163,840-point transonic cloud (640 x 256, 4% jittered, M 0.85, AoA 1 deg,
  CFL 100, one inner iteration, limiter K 5, library-default lanes): residual
  and increment of the free-stream start and of the oracle's state after five
  iterations, and five graph-replayed iterations of ``lskum_solve`` against
  five oracle iterations -- whole fields, FP64 bar 1e-11.
* 2,621,440-point cloud (2560 x 1024, M 0.5, AoA 3 deg): residual and
  increment of the free-stream start, FP64 (1e-11) and mixed precision (1e-4).
"""
import numpy as np
import pytest

import oracle as O
from paper_2406_07441_amd import cloudgen as cg

pytestmark = pytest.mark.gpu

TOL = 1e-11


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def lk():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_07441_amd import lskum
    lskum.lib()
    return lskum


def test_transonic_163840_benchmark_configuration(lk):
    cloud = cg.cloud_163840()
    kw = dict(cfl=100.0, inner_iters=1, limiter=1, limiter_k=5.0)
    o = O.Oracle(cloud, mach=0.85, aoa_deg=1.0, **kw)
    gc = lk.Cloud(cloud)
    assert np.array_equal(gc.colours(), o.colours)
    prm = lk.default_params(check_every=5, tol_rel=0.0, max_iters=5, **kw)
    st = lk.State(gc, 0.85, 1.0, prm)
    U = o.free_stream()
    states = [U]
    for _ in range(5):
        U, _, _, _ = o.iteration(U)
        states.append(U)
    for it in (0, 5):
        st.set_U(states[it])
        R, res = st.residual()
        Ro, reso = o.residual(states[it])
        assert rel(R, Ro) < TOL and abs(res - reso) <= TOL * reso
        st.set_U(states[it])
        st.step()
        _, _, dUo, _ = o.iteration(states[it])
        e = rel(st.get_dU(), dUo)
        print(f"163840 it={it}: dU rel err {e:.3e}")
        assert e < TOL
    # the benchmark's path: graph-replayed iterations from the free stream
    st.set_U(states[0])
    rep = st.solve()
    assert rep.iters == 5
    e = rel(st.get_U(), states[5])
    print(f"163840 five solve iterations: U rel err {e:.3e}")
    assert e < TOL
    st.close()


def test_cloud_2621440_free_stream_step(lk):
    cloud = cg.cloud_2621440()
    o = O.Oracle(cloud, mach=0.5, aoa_deg=3.0, cfl=100.0, inner_iters=1)
    gc = lk.Cloud(cloud)
    U0 = o.free_stream()
    Ro, reso = o.residual(U0)
    _, _, dUo, _ = o.iteration(U0)
    for prec, tol in ((lk.FP64, TOL), (lk.MIXED, 1e-4)):
        st = lk.State(gc, 0.5, 3.0, lk.default_params(cfl=100.0, inner_iters=1, precision=prec))
        R, res = st.residual()
        assert rel(R, Ro) < TOL and abs(res - reso) <= TOL * reso
        st.step()
        e = rel(st.get_dU(), dUo)
        print(f"2621440 precision={prec}: dU rel err {e:.3e}")
        assert e < tol
        st.close()
