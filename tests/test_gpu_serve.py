"""Serving on the device: every simulation's state after the served run is
bitwise the state it reaches alone after the same number of steps (same
kernels, same per-grid dt), through admissions, evictions to host memory and
batches of changing membership on two streams; and a served step matches the
oracle."""
import numpy as np
import pytest

import oracle
from paper_2208_11630_amd import ics

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2208_11630_amd import hydro, serve

    hydro.lib()
    return torch, hydro, serve


def alone_state(torch, hydro, sim, L, k):
    nb = L // 16
    G = hydro.Grid(16, (nb, nb, nb), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (0, 0, 0), 1.4, 1e-10)
    ics.served_state_device(sim, L, out=G.state)
    hydro.lib().hydro_state_changed(G.handle)
    for _ in range(k):
        G.step_cfl(0.8)
    return G.download()


def test_served_states_equal_alone(env):
    torch, hydro, serve = env
    sizes = [32, 48, 32, 64, 48, 32, 64, 32, 48, 32]
    ex = serve.GpuExecutor(sizes)
    budget = 40 * (64 ** 3 + 48 ** 3 + 2 * 32 ** 3) + 4096    # forces evictions
    srv = serve.Server(ex, budget_bytes=budget, max_inflight=2)
    arr = serve.poisson_arrivals(rate=3000, duration=0.05, nsims=len(sizes), seed=6)
    st = srv.run(arr)
    torch.cuda.synchronize()
    s = st.summary()
    print("served:", s, flush=True)
    assert s["completed"] == len(arr)
    assert st.evictions > 0
    # state bytes copied each way: every copy in follows a copy out, and a
    # state is 40 B per cell of whole 16^3 blocks
    assert ex.moved["out"] > 0 and ex.moved["in"] <= ex.moved["out"]
    assert ex.moved["out"] % (40 * 16 ** 3) == 0 and ex.moved["in"] % (40 * 16 ** 3) == 0
    for sim, L in enumerate(sizes):
        k = ex.steps_done[sim]
        got = ex.current_state(sim)
        ref = alone_state(torch, hydro, sim, L, k)
        assert np.array_equal(got, ref), (sim, k)


def test_served_step_matches_oracle(env):
    torch, hydro, serve = env
    L = 48
    sizes = [L]
    ex = serve.GpuExecutor(sizes)
    srv = serve.Server(ex, budget_bytes=10 ** 10)
    ex.make_resident(0)
    U0 = ex.current_state(0).copy()
    srv.used = ex.bytes_of(0)
    srv.lru[0] = None
    st = srv.run([(0.0, 0)])
    torch.cuda.synchronize()
    got = ex.current_state(0)
    nb = L // 16
    P = ics.Problem("srv", 16, (nb, nb, nb), (1.0 / L,) * 3, (0, 0, 0), 1.4, U0)
    g = oracle.Grid(16, P.nb, P.dx, P.bc, P.gamma, P.small_p)
    U = P.U.copy()
    ref, _ = oracle.step(g, U, oracle.dt(g, U, 0.8))
    b = ics.interior(ref, 16)
    for v in range(5):
        den = np.abs(b[:, v]).max() if v in (0, 4) else np.sqrt((b[:, 1:4] ** 2).sum(axis=1)).max()
        assert np.abs(got[:, v] - b[:, v]).max() <= 1e-12 * den
