"""GPU checks of the autotuners through the C ABI: the choice is one of the
candidates, the trial steps leave a consistent state (maintained energy equal
to the exact quotient; b = H c), and a tuned batch still converges to the
oracle ground states within 1e-8 Ha."""
import numpy as np
import pytest

import synth_inputs
from oracle import cd as ocd
from oracle import fci

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2605_04483_amd as api

    return api


def test_tune_k_keeps_a_consistent_state(api):
    h, eri = synth_inputs.ab_initio(10, 30, 5)
    ctx = api.cdfci_init(h, eri, 4, 3, table_slots=1 << 16)
    E_start = api.cdfci_energy(ctx)
    best, rates = api.cdfci_tune_k(ctx, ks=(1, 8, 32), seconds_per_trial=0.01, rounds=2)
    assert best in (1, 8, 32)
    assert all(np.isfinite(v) for v in rates.values())
    E = api.cdfci_energy(ctx)
    assert E < E_start
    assert abs(api.cdfci_energy(ctx, exact=1) - E) < 1e-10 * abs(E)
    ka, kb, c, b = api.cdfci_export(ctx)
    H, basis = ocd.sparse_H(h, eri, 4, 3)
    index = {k: i for i, k in enumerate(basis)}
    cv = np.zeros(len(basis))
    for x, y, v in zip(ka, kb, c):
        cv[index[(int(x), int(y))]] = v
    Hc = H @ cv
    assert max(abs(bv - Hc[index[(int(x), int(y))]]) for x, y, bv in zip(ka, kb, b)) < 1e-10
    ctx.close()


def test_tune_batch_then_converge(api):
    specs = []
    for dims, U in (((2, 2), 2.0), ((2, 3), 5.0), ((2, 4), 4.0), ((6,), 3.0)):
        L = int(np.prod(dims))
        specs.append({"dims": dims, "t": 1.0, "U": U, "n_alpha": (L + 1) // 2, "n_beta": L // 2})
    B = api.cdfci_init_hubbard_batch(specs, dx_threshold=1e-11)
    slots0 = api.cdfci_batch_tables(B)
    chunk, launches, lf = api.cdfci_tune_batch(B, chunks=(128, 1024), launches=(1, 4), load_factors=(0.3, 0.79),
                                               steps_per_trial=2000)
    assert chunk in (128, 1024) and launches in (1, 4) and lf in (0.3, 0.79)
    slots = api.cdfci_batch_tables(B)
    # the tables follow the chosen load factor (larger at 0.3 for the sizes here)
    assert np.all(slots >= slots0) if lf == 0.3 else np.array_equal(slots, slots0)
    for _ in range(10):
        st = api.cdfci_step_batch(B, 500_000)
        print(f"batch: {st}", flush=True)
        if st["running"] == 0:
            break
    E, steps, status = api.cdfci_batch_results(B)
    for i, sp in enumerate(specs):
        h, eri = fci.hubbard_integrals(sp["dims"], sp["t"], sp["U"])
        E0 = ocd.ground_energy(h, eri, sp["n_alpha"], sp["n_beta"])
        assert status[i] == 1
        assert abs(E[i] - E0) < 1e-8
    B.close()
