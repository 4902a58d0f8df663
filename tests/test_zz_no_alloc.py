"""GPU test of cdfci_column_noalloc, the get_column variant that makes no
device allocation (it stages through a fixed device array of the library):
through the C ABI it returns exactly what cdfci_column returns, on two calls
in a row with the second column smaller than the first, into host and device
outputs, and refuses a column above its limit."""
import numpy as np
import pytest

import synth_inputs
from oracle import cd as ocd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2605_04483_amd as api

    return api


def _same(api, ctx, key):
    ka, kb, v = api.cdfci_column(ctx, key)
    na, nb, nv = api.cdfci_column_noalloc(ctx, key)
    assert len(nv) == len(v)
    assert np.array_equal(ka, na) and np.array_equal(kb, nb)
    assert np.array_equal(v.view(np.uint64), nv.view(np.uint64))  # bit for bit
    return len(v)


def test_noalloc_column_equals_column(api):
    import torch

    h36, e36 = synth_inputs.ab_initio(36, 108, synth_inputs.CONFIG_SEEDS["abinitio_n36"])
    big = api.cdfci_init(h36, e36, 8, 8, table_slots=1 << 20)
    h12, e12 = synth_inputs.ab_initio(12, 36, 1)
    small = api.cdfci_init(h12, e12, 5, 4, table_slots=1 << 16, energy_shift=-3.0)
    # first call: a 71,793-entry column; second: a 1,566-entry column
    n1 = _same(api, big, ocd.aufbau(h36, 8, 8))
    n2 = _same(api, small, ocd.aufbau(h12, 5, 4))
    assert (n1, n2) == (71793, 1566)
    # again in the other order, other determinants
    a, b = synth_inputs.random_dets(36, 8, 8, 1, 3)
    _same(api, big, (int(a[0]), int(b[0])))
    a, b = synth_inputs.random_dets(12, 5, 4, 1, 4)
    key = (int(a[0]), int(b[0]))
    _same(api, small, key)
    # device outputs
    kd = torch.zeros(2 * n2, dtype=torch.int64, device="cuda")
    vd = torch.zeros(n2, dtype=torch.float64, device="cuda")
    assert api.cdfci_column_noalloc(small, key, kd, vd) == n2
    ka, kb, v = api.cdfci_column(small, key)
    kk = kd.cpu().numpy().view(np.uint64)
    assert np.array_equal(kk[0::2], ka) and np.array_equal(kk[1::2], kb)
    assert np.array_equal(vd.cpu().numpy(), v)
    big.close()
    small.close()


def test_noalloc_column_above_the_limit(api):
    h, e = synth_inputs.ab_initio(48, 48, 5)
    ctx = api.cdfci_init(h, e, 12, 12, table_slots=1 << 20)
    with pytest.raises(api.CDFCIError) as ei:
        api.cdfci_column_noalloc(ctx, ocd.aufbau(h, 12, 12))
    assert ei.value.code == -2
    ctx.close()
