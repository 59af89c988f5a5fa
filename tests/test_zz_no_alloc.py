"""mgfwa_evaluate_noalloc (fitness without a context or workspace, scratch in a
library-held device array) against the existing entry point mgfwa_evaluate on
a context of the same problem and precision (needs an MI355X).

Two calls in a row per case, the second with fewer rows and a smaller problem,
so stale scratch contents from the first call would show.  FP32 values are
also checked against the oracle's binary64 loss.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2501_03944_amd import inputs
from tests.gpu_util import assert_fitness_close, require_gpu

pytestmark = pytest.mark.gpu

CASES = [
    # (widths, act, loss, samples of the first / second call, rows first / second)
    ((64, 128, 128, 10), "relu", "ce", (1000, 333), (300, 37)),
    ((8, 16, 1), "tanh", "mse", (256, 100), (129, 5)),
    ((784, 256, 10), "relu", "ce", (2000, 700), (64, 20)),     # wide-first-layer kernel
]


def _problem(widths, act, loss, S, seed):
    return inputs.random_mlp_problem(widths, (act,) * (len(widths) - 2), loss, S, seed=seed)


def _noalloc(M, torch, wl, precision, W):
    dev = torch.device("cuda")
    x = torch.from_numpy(wl.x).to(dev)
    y = torch.from_numpy(wl.y).to(dev) if wl.loss == "mse" else None
    lab = torch.from_numpy(wl.labels).to(dev) if wl.loss == "ce" else None
    prob = M.make_problem(wl.widths, wl.acts, wl.loss, wl.x.shape[0], x.data_ptr(),
                          0 if y is None else y.data_ptr(), 0 if lab is None else lab.data_ptr())
    out = torch.full((W.shape[0],), float("nan"), dtype=torch.float32, device=dev)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    M.mgfwa_evaluate_noalloc(prob, M.PRECISION[precision], W.data_ptr(), W.shape[0], W.shape[1],
                             out.data_ptr(), st.cuda_stream)
    st.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("widths,act,loss,samples,rows", CASES)
def test_noalloc_equals_evaluate(widths, act, loss, samples, rows, precision):
    torch, M = require_gpu()
    for call, (S, n) in enumerate(zip(samples, rows)):
        wl = _problem(widths, act, loss, S, seed=40 + call)
        D = wl.dim
        ld = (D + 63) // 64 * 64
        Wh = np.zeros((n, ld), np.float32)
        Wh[:, :D] = inputs.random_weights(D, n, seed=50 + call, lo=-1.0, hi=1.0)
        W = torch.from_numpy(Wh).cuda()
        got = _noalloc(M, torch, wl, precision, W)
        g = M.MGFWA(wl.widths, wl.acts, wl.loss, wl.x, wl.y, wl.labels, n_fireworks=1,
                    n_sparks=2, n_guiding=1, precision=precision)
        want = g.evaluate(W).cpu().numpy()
        g.close()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), \
            f"call {call}: {np.abs(got - want).max()}"
        if precision == "fp32":
            y64 = O.Problem.from_workload(wl).loss_rows(Wh[:, :D])
            assert_fitness_close(got, y64, f"call {call} vs oracle")


def test_noalloc_errors():
    torch, M = require_gpu()
    wl = _problem((64, 128, 128, 10), "relu", "ce", 64, seed=1)
    S = 300_000   # 73 MiB of packed FP32 samples
    big = torch.zeros((S, 64), dtype=torch.float32, device="cuda")
    lab = torch.zeros(S, dtype=torch.int32, device="cuda")
    W = torch.zeros((2, (wl.dim + 63) // 64 * 64), dtype=torch.float32, device="cuda")
    out = torch.zeros(2, dtype=torch.float32, device="cuda")
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    # the packed samples alone exceed the scratch: rejected before any device work
    prob = M.make_problem(wl.widths, wl.acts, "ce", S, big.data_ptr(), 0, lab.data_ptr())
    with pytest.raises(M.MgfwaError) as e:
        M.mgfwa_evaluate_noalloc(prob, M.PRECISION["fp32"], W.data_ptr(), 2, W.shape[1],
                                 out.data_ptr(), st.cuda_stream)
    assert e.value.status == M.EINVAL and "scratch" in str(e.value)
    small = M.make_problem(wl.widths, wl.acts, "ce", 64, big.data_ptr(), 0, lab.data_ptr())
    with pytest.raises(M.MgfwaError) as e:     # the null stream
        M.mgfwa_evaluate_noalloc(small, 0, W.data_ptr(), 2, W.shape[1], out.data_ptr(), 0)
    assert e.value.status == M.EINVAL
    with pytest.raises(M.MgfwaError) as e:     # ld below D
        M.mgfwa_evaluate_noalloc(small, 0, W.data_ptr(), 2, 8, out.data_ptr(), st.cuda_stream)
    assert e.value.status == M.EINVAL
    net = M.make_problem((10, 16, 1), ("relu",), None, 0, net_ptr=W.data_ptr())
    with pytest.raises(M.MgfwaError) as e:     # input problems are not covered
        M.mgfwa_evaluate_noalloc(net, 0, W.data_ptr(), 2, 16, out.data_ptr(), st.cuda_stream)
    assert e.value.status == M.EUNSUPPORTED
    st.synchronize()
