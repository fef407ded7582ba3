"""GPU: the list-stream ceiling diagnostic (rlpt_stream_lists) reads the
sweep's lists and changes nothing of the chain."""
import numpy as np
import pytest

from paper_2511_13508_amd import rlpt
from tests import synth
from tests.gpu_util import make_ctx

pytestmark = pytest.mark.gpu

SEED = 2511135080 + 700


@pytest.mark.parametrize("N,S,T,reps", [(64, 2, 4, 2), (97, 3, 3, 2), (256, 2, 8, 2)])
def test_stream_lists_leaves_the_chain_untouched(N, S, T, reps):
    graphs = [rlpt.Graph(N, SEED + 10 * N + i) for i in range(S)]
    temps = synth.geometric_temps(0.3, 1.5, T)
    kw = dict(n_temps=T, n_reps=reps, precision=rlpt.FP32, swap_interval=1, resync_interval=10,
              measure_start=0, measure_interval=1, n_bins=20, list_layout=rlpt.LAYOUT_CHUNKED)
    a, b = make_ctx(graphs, temps, **kw), make_ctx(graphs, temps, **kw)
    for c in (a, b):
        c.init(4)
        c.sweep(7)
    ms = a.stream_lists(3)
    assert ms > 0.0
    for c in (a, b):
        c.sweep(13)
    assert np.array_equal(a.get_state(), b.get_state())
    assert np.array_equal(a.energies()[0], b.energies()[0])
    oa, ob = a.observables(), b.observables()
    for f in oa:
        assert np.array_equal(oa[f], ob[f]), f
    assert a.counters() == b.counters()


def test_stream_lists_rejects_what_it_does_not_cover():
    g = [rlpt.Graph(32, SEED + 1)]
    temps = synth.geometric_temps(0.5, 1.0, 2)
    c64 = make_ctx(g, temps, n_temps=2, n_reps=1, precision=rlpt.FP64)
    c64.init(1)
    with pytest.raises(rlpt.RlptError) as e:
        c64.stream_lists(1)
    assert e.value.code == rlpt.RLPT_E_UNSUPPORTED
    c32 = make_ctx(g, temps, n_temps=2, n_reps=1, precision=rlpt.FP32, list_layout=rlpt.LAYOUT_CHUNKED)
    with pytest.raises(rlpt.RlptError) as e:
        c32.stream_lists(1)
    assert e.value.code == rlpt.RLPT_E_STATE
