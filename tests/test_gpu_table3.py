"""Table 3 (Sec. 3.3): 2D Burgers, narrow Gaussian, fourth-order convergence.

The kinetic velocity is not given in the paper; V = 3 (sub-characteristic for
u in [0, 1]: w - b u / (2V) > 0 needs V > 2) with N = 128 2^k cells, so that
T / dt = V N / 384 is an integer on every level and the N and 2N runs end at
the same time T = 1/16.  Err-Estim(N) = || u_N - u_2N[::2, ::2] || (discrete L2
with weight dx^2), as in the paper.  The GPU path is checked element-wise
against the oracle on the coarse levels, and its observed order on the fine
levels against 4 (the paper's finest printed order is 3.86).
"""
import numpy as np
import pytest

from conftest import read_golden
from gpu_common import PARITY_RTOL, componentwise_error, to_gpu, to_host

from oracle.lattice import Lattice, grid, steps_for_time, time_step
from oracle.scheme import Relaxer, run
from oracle.systems import Burgers, equilibrium

V = 3.0
T = 1.0 / 16.0
PARAM = (1.0, 0.6)


def gaussian(N):
    x, _ = grid(N)
    X, Y = np.meshgrid(x, x)  # rows are y, columns x
    return np.exp(-100.0 * ((X - 0.5) ** 2 + (Y - 0.5) ** 2))[None]


def gpu_solution(N, relax):
    from paper_2403_13406_amd import Solver
    s = Solver("D2Q4", "burgers", N, N, V=V, relax=relax, param=PARAM)
    f = s.init_equilibrium(to_gpu(gaussian(N)))
    n = s.steps_for_time(T)
    assert n * 24.0 / (V * N) == pytest.approx(T, rel=1e-15)  # lands on T exactly
    s.step(f, n)
    u = s.moments(f)
    s.sync()
    return to_host(u)[0]


def err_estim(coarse, fine):
    N = coarse.shape[0]
    return float(np.sqrt(np.sum((coarse - fine[::2, ::2]) ** 2) / N ** 2))


@pytest.mark.gpu
@pytest.mark.parametrize("relax", ["fixed", "entropic"])
@pytest.mark.parametrize("N", [128, 256])
def test_table3_setup_matches_oracle(N, relax):
    lat, sysb = Lattice("D2Q4"), Burgers(PARAM)
    _, dx = grid(N)
    n = steps_for_time(T, time_step(dx, V))
    want = run(Relaxer(lat, sysb, V, relax), equilibrium(lat, sysb, V, gaussian(N)), n).sum(0)[0]
    got = gpu_solution(N, relax)
    assert max(componentwise_error(got[None, None], want[None, None])) <= PARITY_RTOL


@pytest.mark.gpu
@pytest.mark.parametrize("relax", ["fixed", "entropic"])
def test_table3_fourth_order(relax):
    sols = {N: gpu_solution(N, relax) for N in (512, 1024, 2048, 4096)}
    errs = [err_estim(sols[N], sols[2 * N]) for N in (512, 1024, 2048)]
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    paper_last = float(read_golden("table3_burgers2d_order.txt")[-1][2])
    assert errs[0] > errs[1] > errs[2]
    for p in orders:
        assert 3.5 <= p <= 4.5, orders
        assert abs(p - paper_last) <= 0.4, (orders, paper_last)
