"""Host-side check of the bulge-chasing schedule of the two-stage Casida
eigensolver (csrc/eig2s.hip): step k of sweep i runs at time 2 i + k, all
steps of one time in one launch.  Step (i, k) reads and writes the band
entries of its window (rows i + 1 + k b .. i + (k + 1) b of the previous
window's columns, or column i for k = 0, and the lower triangle of the
diagonal block); this test enumerates those entries and checks, for several
sizes, that the steps of one time never share an entry and that every entry
shared by two steps is reached by the lower sweep first (the order of the
sweep-by-sweep reduction, so the result is the same)."""
import pytest

LAG = 2


def steps(n, b, i):
    return (n - 1 - i + b - 1) // b


def entries(n, b, i, k):
    r0, r1 = i + 1 + k * b, min(i + (k + 1) * b, n - 1)
    if k == 0:
        e = {(r, i) for r in range(r0, r1 + 1)}
    else:
        p0, p1 = i + 1 + (k - 1) * b, min(i + k * b, n - 1)
        e = {(r, c) for r in range(r0, r1 + 1) for c in range(p0, p1 + 1)}
    return e | {(r, c) for r in range(r0, r1 + 1) for c in range(r0, r + 1)}


def schedule(n, b, lag):
    by_t = {}
    for i in range(n - 2):
        for k in range(steps(n, b, i)):
            by_t.setdefault(lag * i + k, []).append((i, k))
    return by_t


@pytest.mark.parametrize("n,b", [(60, 8), (137, 16), (300, 32), (330, 64)])
def test_lag2_steps_of_one_time_are_independent_and_ordered(n, b):
    by_t = schedule(n, b, LAG)
    last = {}
    for t in sorted(by_t):
        seen = set()
        for i, k in by_t[t]:
            e = entries(n, b, i, k)
            assert not (seen & e), (n, b, t, i, k)
            seen |= e
            for x in e:
                assert last.get(x, -1) <= i, (n, b, t, i, k, x)
                last[x] = i


def test_lag1_would_conflict():
    """The check has teeth: with lag 1 two steps of one time share entries."""
    by_t = schedule(60, 8, 1)
    clash = False
    for t in sorted(by_t):
        seen = set()
        for i, k in by_t[t]:
            e = entries(60, 8, i, k)
            clash = clash or bool(seen & e)
            seen |= e
    assert clash


@pytest.mark.parametrize("n,b", [(256, 64), (350, 64), (1001, 64), (10400, 64), (41600, 64), (97, 8)])
def test_sweep_first_step_closed_form(n, b):
    """The first reflector of sweep i sits after the steps of all earlier
    sweeps, sum over i' < i of ceil((n - 1 - i') / b); the kernels compute it
    as S(n - 1) - S(n - 1 - i) with S(x) = b q (q + 1) / 2 + r (q + 1) for
    x = q b + r (the library also checks it against the running sum before
    every bulge chase)."""
    def S(x):
        q, r = divmod(x, b)
        return b * q * (q + 1) // 2 + r * (q + 1)
    run = 0
    for i in range(n - 2):
        assert S(n - 1) - S(n - 1 - i) == run
        run += -(-(n - 1 - i) // b)
