"""Open-ended stepping (mm_batch_begin / mm_batch_advance / mm_batch_end)
through the C ABI: a run advanced in pieces equals one mm_batch_step of the
summed count bit for bit (FSAL, step size and trace carry over between the
pieces; the remainders run as the 16/8/4/2/1-step graphs), on one sequence
and on concurrent sub-batches, and every other call on the batch or its
contexts is refused while the run is open."""
import numpy as np
import pytest

from paper_2603_03706_amd import mmcav, workloads as W
from tests.helpers import gpu_for

pytestmark = pytest.mark.gpu


def _ctxs(insts):
    ctxs = [gpu_for(inst) for inst in insts]
    for c in ctxs:
        c.set_sampling(1e-12, 4000)
    return ctxs


def _snap(ctxs):
    return [(c.get_m(), c.get_a(), c.get_trace(4000), c.stats()["accepted"], c.stats()["rejected"],
             c.stats()["t"], c.stats()["dt"]) for c in ctxs]


def _same(x, y):
    for (m, a, tr, acc, rej, t, dt), (m1, a1, tr1, acc1, rej1, t1, dt1) in zip(x, y):
        assert np.array_equal(m, m1) and np.array_equal(a, a1)
        for u, v in zip(tr, tr1):
            assert np.array_equal(u, v)
        assert (acc, rej, t, dt) == (acc1, rej1, t1, dt1)


@pytest.mark.parametrize("parts", [1, 2])
@pytest.mark.parametrize("method", ["dp45", "rk4"])
def test_advance_in_pieces_equals_one_step_call(parts, method):
    insts = [W.sweep_sphere(k, count=3, n=8 if k % 2 else 12) for k in range(3)]
    for inst in insts:
        inst.method, inst.dt0 = method, (0.2e-12 if method == "rk4" else inst.dt0)
    tol = 1e-6 if method == "dp45" else 0.0
    pieces = [3, 37, 5, 64, 1]              # remainders exercise every small graph

    ref = _ctxs(insts)
    b = mmcav.Batch(ref)
    b.set_streams(parts)
    b.step(sum(pieces), tol)
    want = _snap(ref)
    b.close()

    got_c = _ctxs(insts)
    b = mmcav.Batch(got_c)
    b.set_streams(parts)
    b.begin(tol)
    for k in pieces:
        b.advance(k)
    b.end()
    got = _snap(got_c)
    b.close()
    _same(got, want)
    assert sum(s[3] + s[4] for s in got) == len(insts) * sum(pieces)


def test_open_run_refuses_other_calls():
    insts = [W.sweep_sphere(k, count=2, n=8) for k in range(2)]
    ctxs = _ctxs(insts)
    b = mmcav.Batch(ctxs)
    with pytest.raises(mmcav.MMError) as e:
        b.advance(1)                         # nothing open yet
    assert e.value.status == mmcav.MM_ERR_STATE
    b.begin(1e-6)
    b.advance(4)
    refused = [lambda: ctxs[0].get_m(), lambda: ctxs[0].set_a(np.zeros(1, complex)),
               lambda: ctxs[1].run(1e-12, 1e-6), lambda: ctxs[0].set_sampling(1e-12, 10),
               lambda: b.step(1, 1e-6), lambda: b.run(1e-12, 1e-6), lambda: b.begin(1e-6),
               lambda: mmcav.Batch([ctxs[0]]).begin(1e-6)]
    for call in refused:
        with pytest.raises(mmcav.MMError) as e:
            call()
        assert e.value.status == mmcav.MM_ERR_STATE
    acc4, rej4 = b.counts()                  # read only: allowed in the open run
    assert acc4 + rej4 == 2 * 4
    b.advance(4)
    acc8, rej8 = b.counts()
    b.end()
    assert all(c.stats()["accepted"] + c.stats()["rejected"] == 8 for c in ctxs)
    assert (acc8, rej8) == (sum(c.stats()["accepted"] for c in ctxs), sum(c.stats()["rejected"] for c in ctxs))
    ctxs[0].get_m()                          # usable again
    b.begin(1e-6)
    b.close()                                # destroy waits and closes the open run
    ctxs[0].get_m()
