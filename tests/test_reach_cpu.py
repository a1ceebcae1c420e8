"""Pins the reach table used by the maximum-extent backward test: a change of
one stage's value at one pixel (a ReLU or max-pool decision flipping) can
alter only visibility pixels within that stage's reach of its level-0
footprint, so a visibility gradient outside that reach never passes through
the decision.  Checked with the float64 oracle's own stage functions on a
64 x 64 image: every output pixel beyond the reach must be bit-identical."""
import numpy as np
import pytest

import nsm_synth as S
from oracle import net as onet
from test_gpu_backward import REACH, _rand


def _forward(P, x, hit):
    """The U3 forward (oracle stage functions) with `hit(name, tensor)` applied
    to each stage's value before it is used further."""
    z = hit("E0", onet.conv3x3(x, *P["E0"]))
    a0 = onet.relu(z)
    p0 = hit("pool0", onet.maxpool2(a0))
    a1 = onet.relu(hit("E1", onet.conv3x3(p0, *P["E1"])))
    p1 = hit("pool1", onet.maxpool2(a1))
    b = onet.relu(hit("B", onet.conv3x3(p1, *P["B"])))
    d1 = onet.relu(hit("D1", onet.conv3x3(np.concatenate([a1, onet.upsample2(b)], -1), *P["D1"])))
    d0 = onet.relu(hit("D0", onet.conv3x3(np.concatenate([a0, onet.upsample2(d1)], -1), *P["D0"])))
    wh, bh = P["H"]
    return d0 @ wh[0, 0, 0, :] + bh[0]


LEVEL = {"E0": 0, "D0": 0, "E1": 1, "D1": 1, "pool0": 1, "B": 2, "pool1": 2}


@pytest.mark.parametrize("name", sorted(LEVEL))
def test_decision_reach(name):
    assert S.U3.widths == (16, 32, 64)
    flat = S.he_weights(S.U3, 31, bias_scale=0.1)
    P = onet.split_params(6, S.U3.widths, flat)
    x = _rand((1, 64, 64, 6), 32).astype(np.float64)
    base = _forward(P, x, lambda n, t: t)
    l = LEVEL[name]
    worst = 0
    for q in [(0, 0), (5, 9), (7, 3), ((64 >> l) - 1, (64 >> l) - 1)]:
        def hit(n, t, q=q):
            if n != name:
                return t
            t = t.copy()
            t[0, q[0], q[1], :] += 3.0 * (np.abs(t).max() + 1.0)
            return t
        diff = _forward(P, x, hit) != base
        ys, xs = np.nonzero(diff[0])
        assert len(ys) > 0
        lo_y, hi_y = q[0] << l, ((q[0] + 1) << l) - 1
        lo_x, hi_x = q[1] << l, ((q[1] + 1) << l) - 1
        reach = max(np.maximum(lo_y - ys, ys - hi_y).max(), np.maximum(lo_x - xs, xs - hi_x).max(), 0)
        worst = max(worst, int(reach))
    print(f"{name}: measured reach {worst}, table {REACH[name]}")
    assert worst <= REACH[name]
