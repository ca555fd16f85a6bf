"""GPU tests of schedules and the tuner: every schedule the tuner may choose
(plain plans and the batch kernel) matches the FP64 oracle; tuning picks a
schedule no slower than the planner's rule and later plans use it; the
table saved after tuning reloads to the same choices."""
import numpy as np
import pytest

import siggen
from parity import assert_close, spectrum_rms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture
def dd():
    import paper_2403_16665_amd as m
    m.dense_dft_tune_clear()
    yield m
    m.dense_dft_tune_clear()


def inputs(code, N, batch, seed):
    import paper_2403_16665_amd as m
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(batch):
        if code in (m.DD_F32, m.DD_F64):
            x = rng.standard_normal(N)
            rows.append(x.astype(np.float32 if code == m.DD_F32 else np.float64))
        else:
            x = siggen.tones_complex(rng, N, 1e-3)
            rows.append(x if code == m.DD_C64 else x.astype(np.complex128))
    return np.stack(rows)


@pytest.mark.parametrize("N,alpha,batch,code", [
    (1024, 16, 1, 1), (4096, 4, 2, 0), (3 * 2 ** 15, 3, 2, 1), (1024, 4, 1, 2), (65536, 8, 3, 1),
    (5 * 2 ** 12, 2, 2, 3), (256, 8, 37, 1), (320, 3, 13, 0), (48, 5, 29, 1)])
def test_every_plan_schedule_matches_oracle(dd, oracle_mod, N, alpha, batch, code):
    import torch
    x = inputs(code, N, batch, 11)
    xd = torch.from_numpy(x).cuda()
    T = N * 1e-3
    rng = np.random.default_rng(3)
    bins = siggen.bin_subset(rng, alpha * N, 192)
    refs = [oracle_mod.alpha_dft_bins(x[b], alpha, T, bins) for b in range(batch)]
    kind = "f64" if code in (dd.DD_F64, dd.DD_C128) else "f32"
    cands = dd.dense_dft_sched_candidates(N, alpha, batch, code)
    assert len(cands) >= 2
    for sc in cands:
        plan = dd.dense_dft_plan_sched(N, alpha, T, batch, code, sc)
        got = dd.dense_dft_plan_get_sched(plan)
        assert got == sc.as_dict()
        X = dd.alpha_dft(xd, alpha, T, plan=plan).cpu().numpy()
        for b in range(batch):
            assert_close(X[b][bins], refs[b], kind, f"schedule {sc.as_dict()} signal {b}",
                         full_rms=spectrum_rms(x[b], T))


@pytest.mark.parametrize("N,alpha", [(65536, 8), (1024, 16), (3072, 4), (320, 2), (5 * 2 ** 13, 3)])
def test_every_batch_schedule_matches_oracle(dd, oracle_mod, N, alpha):
    import torch
    x = inputs(dd.DD_C64, N, 3, 12)
    xs = [torch.from_numpy(r).cuda() for r in x]
    T = N * 1e-3
    rng = np.random.default_rng(4)
    bins = siggen.bin_subset(rng, alpha * N, 192)
    refs = [oracle_mod.alpha_dft_bins(r, alpha, T, bins) for r in x]
    for sc in dd.dense_dft_batch_sched_candidates(N, alpha):
        Xs = [torch.zeros(alpha * N, dtype=torch.complex64, device="cuda") for _ in xs]
        torch.cuda.synchronize()
        b = dd.dense_dft_batch_plan_sched([(N, alpha, T, dd.DD_C64, xs[i], Xs[i]) for i in range(3)], sc)
        dd.dense_dft_batch_exec(b)
        torch.cuda.synchronize()
        for i in range(3):
            assert_close(Xs[i].cpu().numpy()[bins], refs[i], "f32", f"batch schedule {sc.as_dict()}",
                         full_rms=spectrum_rms(x[i], T))


def test_tune_plan_and_reload(dd, tmp_path):
    info = dd.dense_dft_tune(1024, 16, 1, dd.DD_C64)
    assert info["candidates"] >= 2
    assert 0 < info["ms_best"] <= info["ms_default"] * 1.0001
    plan = dd.dense_dft_plan(1024, 16, 1.024, 1, dd.DD_C64)
    assert dd.dense_dft_plan_get_sched(plan) == info["best"]
    info2 = dd.dense_dft_tune(65536, 8, 8, dd.DD_C64)
    assert info2["ms_best"] <= info2["ms_default"] * 1.0001
    binfo = dd.dense_dft_tune_batch(1024, 16)
    assert binfo["candidates"] >= 1 and binfo["ms_best"] > 0
    path = tmp_path / "tuned.txt"
    dd.dense_dft_tune_save(str(path))
    dd.dense_dft_tune_clear()
    dd.dense_dft_tune_load(str(path))
    assert dd.dense_dft_tune_entries() == (2, 1)
    plan = dd.dense_dft_plan(1024, 16, 1.024, 1, dd.DD_C64)
    assert dd.dense_dft_plan_get_sched(plan) == info["best"]


@pytest.mark.parametrize("N,alpha,batch,code", [(256, 8, 37, 1), (384, 3, 13, 0), (1024, 4, 5, 3)])
def test_every_one_pass_schedule_round_trips(dd, N, alpha, batch, code):
    # the inverse runs the forward's block shape: each group sums its values
    # of j, and the groups' partial sums meet in LDS
    import torch
    x = inputs(code, N, batch, 5)
    xd = torch.from_numpy(x).cuda()
    T = N * 1e-3
    cands = [sc for sc in dd.dense_dft_sched_candidates(N, alpha, batch, code) if sc.passes == 1]
    assert len(cands) >= 2
    tol = 1e-12 if code in (dd.DD_F64, dd.DD_C128) else 1e-5
    for sc in cands:
        plan = dd.dense_dft_plan_sched(N, alpha, T, batch, code, sc)
        X = dd.alpha_dft(xd, alpha, T, plan=plan)
        back = torch.empty((batch, N), dtype=X.dtype, device="cuda")
        dd.dense_dft_exec_inverse(plan, X, back)
        torch.cuda.synchronize()
        back = back.cpu().numpy()
        for b in range(batch):
            ref = x[b].astype(back.dtype)
            r = np.linalg.norm(back[b] - ref) / np.linalg.norm(ref)
            assert r <= tol, f"schedule {sc.as_dict()} signal {b}: round trip rel L2 {r:.3e}"
