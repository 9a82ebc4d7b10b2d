"""Why the extrapolator-corrector subtracts the previous extrapolation (paper
Sec. 2.4).  The paper writes the estimate as the previous step's actual
source, minus the previous step's estimate, plus the new extrapolation, and
states that subtracting the previous estimate makes the procedure
conservative over time.  Taken literally, with the whole previous estimate
(its own corrector included) subtracted, the recursion is neither
conservative nor convergent: for a constant actual source the zero
extrapolator applies S, 0, S, 0, ... (half the source is lost) and the
constant one 2S, 0, 2S, 0, ... for ever.  Subtracting only the part of the
previous estimate that stood in for the then unknown source, its
extrapolation, makes the applied sources telescope to the actual ones plus
the one extrapolation outstanding, and makes the zero extrapolator apply
each source unchanged one step late, as the paper describes it.  This test
shows both properties on a constant source; the oracle and the kernels use
the second reading."""
import numpy as np


def _literal(kind, S, n):
    est, applied = 0.0, []
    for k in range(n):
        last = S if k > 0 else 0.0
        prev2 = S if k > 1 else 0.0
        ext = [0.0, last, 2 * last - prev2][kind]
        est = last - est + ext
        applied.append(est)
    return np.array(applied)


def _corrector_of_extrapolation(kind, S, n):
    ext_prev, applied = 0.0, []
    for k in range(n):
        last = S if k > 0 else 0.0
        prev2 = S if k > 1 else 0.0
        ext = [0.0, last, 2 * last - prev2][kind]
        applied.append(last - ext_prev + ext)
        ext_prev = ext
    return np.array(applied)


def test_literal_recursion_is_not_conservative():
    n, S = 40, 1.0
    lit0, lit1 = _literal(0, S, n), _literal(1, S, n)
    assert np.allclose(lit0[1:7], [1, 0, 1, 0, 1, 0])     # half of the source lost
    assert np.allclose(lit1[1:7], [2, 0, 2, 0, 2, 0])     # oscillates for ever
    assert abs(lit0.sum() - (n - 1) * S) > 0.4 * n


def test_corrector_of_extrapolation_is_conservative():
    n, S = 40, 1.0
    for kind in (0, 1, 2):
        a = _corrector_of_extrapolation(kind, S, n)
        outstanding = [0.0, S, S][kind]
        assert np.isclose(a.sum(), (n - 1) * S + outstanding)
        assert np.allclose(a[3:], S)                       # settles on the source
