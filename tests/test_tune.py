"""The autotuner's selection rule (paper_2210_17093_amd/tune.py) on the CPU,
with a stand-in timer: a candidate table is kept only if the energies it
gives stay within a rounding-order difference of the default table's (1e-10
Ha for FP64), the fastest kept value of each key wins, and joint keys set
both of their entries."""
import numpy as np
import pytest

pytest.importorskip("torch")
import paper_2210_17093_amd.tune as T  # noqa: E402


class FakeCtx:
    closed = False

    def close(self):
        self.closed = True


def fake_timer(bad=(), slow=None):
    """run(spec): every kernel 1 ms, plus 1 ms per entry that differs from the
    default table (so the defaults win unless `slow` makes them slower);
    energies moved by 1e-6 Ha for the (key, value) pairs in `bad`."""
    slow = slow or {}
    base = np.linspace(-1.0, 1.0, 7)

    def run(spec):
        table = dict(kv.split("=") for kv in spec.split(","))
        extra = sum(1 for k, v in table.items() if str(T.DEFAULTS[k]) != v)
        extra += sum(slow.get((k, v), 0.0) for k, v in table.items())
        ms = {k: 1.0 + extra for k in ("mo_transform_1", "mo_transform_2", "casida",
                                       "residue_rho", "residue_w", "sigma_qs_gemm",
                                       "sigma_qs_reduce", "fock")}
        moved = any((k, v) in bad for k, v in table.items())
        return ms, base + (1e-6 if moved else 0.0)
    ctx = FakeCtx()
    return ctx, run


def test_defaults_win_when_nothing_is_faster():
    ctx, run = fake_timer()
    out = T.tune("cfg3", reps=1, timer=(ctx, run))
    assert out["spec"] == T.spec_of(T.DEFAULTS)
    assert ctx.closed


def test_fastest_kept_value_wins_and_moved_energies_are_dropped():
    # make the default mo1 slow, and the fastest alternative move the energies
    slow = {("mo1", "128x64"): 5.0, ("mo1", "128x128"): 0.0}
    ctx, run = fake_timer(bad={("mo1", "64x64")}, slow=slow)
    out = T.tune("cfg3", reps=1, timer=(ctx, run))
    got = dict(kv.split("=") for kv in out["spec"].split(","))
    assert got["mo1"] == "128x128"  # 64x64 would be as fast but moves the energies
    assert not any(t["key"] == "mo1" and t["value"] == "64x64" for t in out["trials"])


def test_joint_key_sets_both_entries():
    table = dict(T.DEFAULTS)
    T.assign(table, "sigma+sigma_target", "128x128+65536")
    assert table["sigma"] == "128x128" and table["sigma_target"] == "65536"
