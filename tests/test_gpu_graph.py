"""Plain executions captured in HIP graphs: forward (complex and real input,
one and two passes, a ragged chunk) and inverse.  Each graph is replayed
several times with new samples written into the captured input buffer and
eager work between replays; every replay must equal an eager execution of the
same plan bit for bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def fill(x, gen):
    import torch
    n = x.numel()
    if x.is_complex():
        v = (gen.standard_normal(n) + 1j * gen.standard_normal(n)).astype(
            np.complex64 if x.dtype == torch.complex64 else np.complex128)
    else:
        v = gen.standard_normal(n).astype(np.float32 if x.dtype == torch.float32 else np.float64)
    x.copy_(torch.from_numpy(v.reshape(x.shape)).cuda())


@pytest.mark.parametrize("N,alpha,batch,code", [
    (65536, 8, 35, 1),    # two passes, two chunks, the second ragged
    (65536, 8, 35, 0),    # the same, real input (Hermitian half rows)
    (1024, 4, 5, 0),      # one pass, real input
    (3 * 2 ** 12, 5, 3, 3),  # two passes, complex128
])
def test_exec_graph_replay(N, alpha, batch, code):
    import torch
    import paper_2403_16665_amd as dd
    T = N * 1e-3
    plan = dd.dense_dft_plan(N, alpha, T, batch, code)
    in_dtype = {dd.DD_F32: torch.float32, dd.DD_C64: torch.complex64, dd.DD_F64: torch.float64,
                dd.DD_C128: torch.complex128}[code]
    x = torch.empty((batch, N), dtype=in_dtype, device="cuda")
    X = torch.zeros((batch, alpha * N), dtype=dd.out_dtype(code), device="cuda")
    ref = torch.zeros_like(X)
    fill(x, np.random.default_rng(1))
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        dd.dense_dft_exec(plan, x, X, stream=torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        fill(x, np.random.default_rng(10 + rep))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        dd.dense_dft_exec(plan, x, ref)
        torch.cuda.synchronize()
        assert torch.equal(X, ref), f"replay {rep} differs from eager"
        X.zero_()   # eager work between replays


def test_inverse_graph_replay():
    import torch
    import paper_2403_16665_amd as dd
    N, alpha, batch, T = 65536, 4, 3, 1.0
    plan = dd.dense_dft_plan(N, alpha, T, batch, dd.DD_C64)
    Xs = torch.empty((batch, alpha * N), dtype=torch.complex64, device="cuda")
    x = torch.zeros((batch, N), dtype=torch.complex64, device="cuda")
    ref = torch.zeros_like(x)
    fill(Xs, np.random.default_rng(2))
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        dd.dense_dft_exec_inverse(plan, Xs, x, stream=torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        fill(Xs, np.random.default_rng(20 + rep))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        dd.dense_dft_exec_inverse(plan, Xs, ref)
        torch.cuda.synchronize()
        assert torch.equal(x, ref), f"replay {rep} differs from eager"
        x.zero_()


def test_plan_object_api(oracle_mod):
    """plan(...).exec(x) and .exec_inverse(X) with torch dtypes: the same
    results as the function API, and a round trip back to the samples."""
    import torch
    import paper_2403_16665_amd as dd
    from parity import assert_close
    rng = np.random.default_rng(5)
    N, alpha, T = 4096, 4, 2.0
    x = torch.from_numpy((rng.standard_normal((2, N)) + 1j * rng.standard_normal((2, N))).astype(np.complex64)).cuda()
    p = dd.plan(N, alpha, T, 2, torch.complex64)
    X = p.exec(x)
    assert X.shape == (2, alpha * N) and X.dtype == torch.complex64
    ref = dd.alpha_dft(x, alpha, T)
    torch.cuda.synchronize()
    assert torch.equal(X, ref)
    back = p.exec_inverse(X)
    torch.cuda.synchronize()
    assert_close(back[0].cpu().numpy(), x[0].cpu().numpy(), "f32", "round trip")
    pd = dd.dense_dft_plan_decimated(N, 4, T, 2, dd.DD_C64)
    assert pd.M == N // 4
    assert torch.equal(pd.exec(x), dd.decimated_dft(x, 4, T))
