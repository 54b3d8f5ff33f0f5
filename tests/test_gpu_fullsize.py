"""Parity at the benchmark sizes, in the launch configuration the benchmark times.

* 163,840-point transonic cloud (640 x 256, 4% jittered, M 0.85, AoA 1 deg,
  CFL 100, one inner iteration, limiter K 5, library-default lanes): residual
  and increment of the free-stream start and of the oracle's state after five
  iterations, and five graph-replayed iterations of ``lskum_solve`` against
  five oracle iterations -- whole fields, FP64 bar 1e-11.
* 2,621,440-point cloud (2560 x 1024, M 0.5, AoA 3 deg, the benchmark's timed
  workload: CFL 100, one inner iteration, limiter K 5): the GPU's own FP64
  states after 0, 1 and 10 graph-replayed iterations loaded into the oracle,
  residual, increment and new state of the next iteration (FP64 bar 1e-11,
  per component); mixed precision against the FP64 oracle (1e-4).
"""
import numpy as np
import pytest

import oracle as O
from paper_2406_07441_amd import cloudgen as cg

pytestmark = pytest.mark.gpu

TOL = 1e-11


def rel(a, b):
    """Largest error relative to the reference's magnitude, per component."""
    scale = np.abs(b).max()
    return float(max(np.abs(a[v] - b[v]).max() / (np.abs(b[v]).max() or scale)
                     for v in range(b.shape[0])))


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


def test_cloud_2621440_benchmark_configuration(lk):
    # the timed workload of the benchmark: FP64 states after 0, 1 and 10
    # graph-replayed GPU iterations are loaded into the oracle; the residual and
    # the next iteration's increment and state must agree
    cloud = cg.cloud_2621440()
    kw = dict(cfl=100.0, inner_iters=1, limiter=1, limiter_k=5.0)
    o = O.Oracle(cloud, mach=0.5, aoa_deg=3.0, **kw)
    gc = lk.Cloud(cloud)
    assert np.array_equal(gc.colours(), o.colours)
    prm = lk.default_params(check_every=1, tol_rel=0.0, max_iters=1, **kw)
    st = lk.State(gc, 0.5, 3.0, prm)
    states = {0: st.get_U()}
    assert rel(states[0], o.free_stream()) < 1e-14
    st.solve()
    states[1] = st.get_U()
    prm.max_iters = 9
    st.set_params(prm)
    st.solve()
    states[10] = st.get_U()
    dUo10 = None
    for it in (0, 1, 10):
        U = states[it]
        st.set_U(U)
        R, res = st.residual()
        Ro, reso = o.residual(U)
        st.set_U(U)
        st.step()
        Un, _, dUo, _ = o.iteration(U)
        e = (rel(R, Ro), rel(st.get_dU(), dUo), rel(st.get_U() - U, Un - U))
        print(f"2621440 GPU state after {it} iterations: R {e[0]:.2e} dU {e[1]:.2e} "
              f"U change {e[2]:.2e}", flush=True)
        assert max(e) < TOL and abs(res - reso) <= TOL * reso
        dUo10 = dUo
    st.close()
    mx = lk.State(gc, 0.5, 3.0, lk.default_params(precision=lk.MIXED, **kw))
    mx.set_U(states[10])
    mx.step()
    e = rel(mx.get_dU(), dUo10)
    print(f"2621440 mixed precision, state after 10 iterations: dU rel err {e:.3e}")
    assert e < 1e-4
    mx.close()
