"""Tuner and schedule checks that need no GPU: candidate schedules are valid
splits and start with the planner's choice; bad schedules are refused; the
tuning table round-trips through its text file, is consulted by the planner
and by the batch scheduler, and is read from DD_TUNE_DB."""
import ctypes
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture
def dd():
    import paper_2403_16665_amd as m
    m.dense_dft_tune_clear()
    yield m
    m.dense_dft_tune_clear()


@pytest.mark.parametrize("N,alpha,batch,dtype", [
    (65536, 8, 256, 1), (1024, 16, 1, 1), (1 << 22, 16, 1, 1), (1024, 4, 1, 2), (98304, 3, 4, 0),
    (320, 2, 8, 0), (5 * 2 ** 14, 16, 2, 3)])
def test_candidates_are_valid_schedules(dd, N, alpha, batch, dtype):
    c = dd.dense_dft_sched_candidates(N, alpha, batch, dtype)
    assert len(c) >= 1
    keys = set()
    for s in c:
        assert s.passes in (1, 2)
        assert s.N1 * s.N2 == N
        if s.passes == 1:
            # lines signals per block, jgroup thread groups per signal
            assert s.N2 == 1 and 1 <= s.lines <= batch and 1 <= s.jgroup <= alpha
        else:
            assert 1 <= s.jgroup <= alpha and 1 <= s.chunk <= batch and s.N2 & (s.N2 - 1) == 0
        keys.add((s.passes, s.lines, s.N1, s.N2, s.jgroup, s.chunk))
    assert len(keys) == len(c)  # no duplicates


@pytest.mark.parametrize("sched", [
    dict(passes=3), dict(passes=2, N1=100, N2=64), dict(passes=2, N1=256, N2=256, jgroup=9),
    dict(passes=2, N1=8192, N2=8), dict(passes=1, N1=65536, N2=1), dict(passes=2, N1=4096, N2=16, jgroup=-1),
    dict(passes=2, N1=2, N2=32768)])
def test_plan_sched_refuses_bad_schedules(dd, sched):
    h = ctypes.c_void_p(3)
    sc = dd.make_sched(**sched)
    assert dd._lib.dense_dft_plan_sched(ctypes.byref(h), 65536, 8, 1.0, 4, dd.DD_C64, 0, ctypes.byref(sc)) == 2
    assert not h.value
    assert dd._lib.dense_dft_plan_sched(ctypes.byref(h), 65536, 8, 1.0, 4, dd.DD_C64, 0, None) == 1


@pytest.mark.parametrize("lines,jgroup", [(1, 5), (4, 4), (2, 3), (-1, 1), (1, -2)])
def test_plan_sched_refuses_bad_one_pass_shapes(dd, lines, jgroup):
    # N = 1024 runs 64 threads per line, 4 lines per block: lines * jgroup <= 4, jgroup <= alpha
    h = ctypes.c_void_p(3)
    sc = dd.make_sched(passes=1, N1=1024, N2=1, lines=lines, jgroup=jgroup)
    assert dd._lib.dense_dft_plan_sched(ctypes.byref(h), 1024, 4, 1.0, 8, dd.DD_C64, 0, ctypes.byref(sc)) == 2
    assert not h.value


def test_one_pass_rule_shares_signals_between_groups(dd):
    # the planner's one-pass shape: every value of j of a signal in one round
    # where the block holds them (complex input: alpha values; real: alpha/2 + 1)
    for N, alpha, batch, dtype, groups in [(1024, 4, 1, dd.DD_F32, 3), (1024, 4, 64, dd.DD_C64, 4),
                                           (256, 8, 4096, dd.DD_C64, 8), (64, 16, 100, dd.DD_C64, 16)]:
        s = dd.dense_dft_sched_candidates(N, alpha, batch, dtype)[0]
        assert (s.passes, s.jgroup) == (1, groups)


def test_batch_candidates(dd):
    for N, a in [(65536, 8), (1024, 16), (3072, 4), (262144, 16), (320, 2), (256, 2)]:
        c = dd.dense_dft_batch_sched_candidates(N, a)
        assert c and all(s.N1 * s.N2 == N and s.passes in (1, 2) for s in c)
    with pytest.raises(dd.DenseDFTError):
        dd.dense_dft_batch_sched_candidates(7, 2)


TABLE = """# hand-written tuning table
plan 1024 16 0 0 2 0 32 32 4 1 0.05
plan 65536 8 0 8 2 0 512 128 8 32 0.6
batch 1024 16 2 16 64 0.001
batch 3072 4 2 24 128 0.002
plan garbage line
batch 10 10
plan 1024 16 0 0 7 0 32 32 4 1 0.05
"""


def test_table_load_save_clear_and_planner_use(dd, tmp_path):
    src = tmp_path / "in.txt"
    src.write_text(TABLE)
    dd.dense_dft_tune_load(str(src))
    # each "plan" line (keyed by precision) serves both input dtypes of it
    assert dd.dense_dft_tune_entries() == (4, 2)
    # the planner's choice (first candidate) is now the table's schedule
    first = dd.dense_dft_sched_candidates(1024, 16, 1, dd.DD_C64)[0]
    assert (first.passes, first.N1, first.N2, first.jgroup) == (2, 32, 32, 4)
    first = dd.dense_dft_sched_candidates(65536, 8, 256, dd.DD_C64)[0]   # batch class 8 = 256..511
    assert (first.N1, first.N2, first.jgroup, first.chunk) == (512, 128, 8, 32)
    other = dd.dense_dft_sched_candidates(65536, 8, 16, dd.DD_C64)[0]    # another batch class: rule
    assert (other.N1, other.N2) == (256, 256)
    out = tmp_path / "out.txt"
    dd.dense_dft_tune_save(str(out))
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert len(lines) == 6 and sum(l.startswith("plan2 ") for l in lines) == 4
    dd.dense_dft_tune_clear()
    assert dd.dense_dft_tune_entries() == (0, 0)
    dd.dense_dft_tune_load(str(out))
    assert dd.dense_dft_tune_entries() == (4, 2)
    with pytest.raises(dd.DenseDFTError):
        dd.dense_dft_tune_load(str(tmp_path / "missing.txt"))


def test_table_from_environment(tmp_path):
    src = tmp_path / "db.txt"
    src.write_text(TABLE)
    code = ("import paper_2403_16665_amd as dd; "
            "print(dd.dense_dft_tune_entries()); "
            "s = dd.dense_dft_sched_candidates(1024, 16, 1, dd.DD_C64)[0]; print(s.N1, s.N2, s.jgroup)")
    env = dict(os.environ, DD_TUNE_DB=str(src))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, env=env,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split("\n")[:2] == ["(4, 2)", "32 32 4"]


def test_table_entries_per_input_dtype(dd, tmp_path):
    """A plan2 entry is keyed by input dtype: it serves real float32 plans of
    its class and leaves complex64 plans of the same class to the rule."""
    src = tmp_path / "v2.txt"
    src.write_text("plan2 65536 8 0 8 2 0 512 128 8 32 0.6\n")
    dd.dense_dft_tune_load(str(src))
    assert dd.dense_dft_tune_entries() == (1, 0)
    real = dd.dense_dft_sched_candidates(65536, 8, 256, dd.DD_F32)[0]
    cplx = dd.dense_dft_sched_candidates(65536, 8, 256, dd.DD_C64)[0]
    assert (real.N1, real.N2) == (512, 128)
    assert (cplx.N1, cplx.N2) == (256, 256)


def test_tune_null_arguments(dd):
    assert dd._lib.dense_dft_tune(1024, 4, 1, 1, None) == 1
    assert dd._lib.dense_dft_tune_batch(1024, 4, None) == 1
    assert dd._lib.dense_dft_tune_save(None) == 1
    assert dd._lib.dense_dft_tune_load(None) == 1
    n = ctypes.c_int32()
    assert dd._lib.dense_dft_sched_candidates(1024, 4, 1, 1, None, 4, ctypes.byref(n)) == 1
    assert dd._lib.dense_dft_sched_candidates(7, 4, 1, 1, None, 0, ctypes.byref(n)) == 2
