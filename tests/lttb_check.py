"""Step-wise LTTB parity rule.

The GPU's pick at step k may differ from the oracle's only where the two
areas are a near tie: for each step, the oracle re-runs that step from the
GPU's previous pick (so one legitimate divergence does not cascade) and the
GPU's pick is accepted if it equals the oracle's, or if its doubled area is
within 1e-12 relative of the oracle's maximum.  Returns the number of
near-tie acceptances (0 means the walk is identical step by step)."""
import numpy as np

REL = 1e-12


def stepwise_check(oracle_mod, y, n_out, got, x=None, sel=None):
    got = np.asarray(got, np.int64)
    m = len(y) if sel is None else len(sel)
    if m <= n_out:
        assert np.array_equal(got, np.arange(m) if sel is None else np.asarray(sel)), "must keep all"
        return 0
    assert len(got) == n_out and got[0] == (0 if sel is None else sel[0])
    pos_of = (lambda s: int(s)) if sel is None else {int(v): i for i, v in enumerate(sel)}.__getitem__
    near = 0
    for k in range(n_out - 2):
        a = pos_of(got[k])
        b = pos_of(got[k + 1])
        pick, best, mine = oracle_mod.lttb_step(y, n_out, k, a, b, x=x, sel=sel)
        if pick == b:
            continue
        assert best > 0 and best - mine <= REL * best, (k, pick, b, best, mine)
        near += 1
    assert got[-1] == (m - 1 if sel is None else sel[-1])
    return near
