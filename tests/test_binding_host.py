"""Host side of the Python binding (no GPU): the per-solve statistics come back
as one numpy structured array with the C struct's fields."""
import numpy as np

from paper_2311_13862_amd import rbws


def test_stats_array_fields_and_copy():
    st = (rbws.SolveStat * 5)()
    for b in range(5):
        st[b].iters = 10 + b
        st[b].outer_iters = b
        st[b].status = rbws.SOLVE_CONVERGED if b != 3 else rbws.SOLVE_MAXITER
        st[b].final_rr = 1e-20 * (b + 1)
        st[b].ff = 2.0
    a = rbws.stats_array(st, 4)
    assert len(a) == 4
    assert set(n for n, _ in rbws.SolveStat._fields_) == set(a.dtype.names)
    assert list(a["iters"]) == [10, 11, 12, 13]
    assert a[3]["status"] == rbws.SOLVE_MAXITER and a[2]["status"] == rbws.SOLVE_CONVERGED
    assert np.allclose(np.sqrt(a["final_rr"] / a["ff"]), np.sqrt(1e-20 * np.arange(1, 5) / 2.0))
    st[0].iters = 99  # the array is a copy, not a view of the C buffer
    assert a[0]["iters"] == 10
    assert all(int(s["outer_iters"]) == b for b, s in enumerate(a))
