"""The allocation-free batched solve (wob_solve_batched_static, through the C
ABI) against the allocating one-shot batched solve (wob_solve_batched): two
calls in a row, the second with fewer problems and fewer points, each
bitwise equal to the allocating solve of the same problems."""
import numpy as np
import pytest

from tests.test_gpu_batch import small_problems

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def W():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_04403_amd import wob
    wob.lib()
    return wob


def _fresh(outs):
    for m, v in outs:
        m.fill_(float("nan"))
        if v is not None:
            v.fill_(float("nan"))


def test_static_batched_solve_equals_allocating_solve(W):
    probs = small_problems(W)
    # call 1: every problem (interior Dirichlet and exterior Neumann, N 64..512)
    ref = W.solve_batched(probs)
    got = W.solve_batched(probs, no_alloc=True)
    torch.cuda.synchronize()
    for (m, v), (mr, vr) in zip(got, ref):
        assert torch.isfinite(mr).all()
        assert torch.equal(m, mr) and torch.equal(v, vr)
    # call 2: fewer problems, fewer points, caller-owned outputs; the array
    # keeps call 1's table, which call 2 overwrites
    small = []
    for k in (2, 0):
        p = dict(probs[k])
        p["points"] = p["points"][:37].contiguous()
        p["mean_out"] = torch.empty(37, dtype=torch.float32, device="cuda")
        p["var_out"] = torch.empty(37, dtype=torch.float32, device="cuda")
        small.append(p)
    got2 = W.solve_batched(small, no_alloc=True)
    outs2 = [(p["mean_out"].clone(), p["var_out"].clone()) for p in small]
    for p in small:
        p["mean_out"], p["var_out"] = None, None
    ref2 = W.solve_batched(small)
    torch.cuda.synchronize()
    for (m, v), (mo, vo), (mr, vr) in zip(got2, outs2, ref2):
        assert torch.equal(m, mo) and torch.equal(v, vo)
        assert torch.equal(m, mr) and torch.equal(v, vr)
        # and the same points of the first call (paths depend on the point index only)
    assert torch.equal(got2[1][0], ref[0][0][:37])
    # a given launch shape
    got3 = W.solve_batched(probs[:3], tune=(128, 2), no_alloc=True)
    ref3 = W.solve_batched(probs[:3], tune=(128, 2))
    torch.cuda.synchronize()
    for (m, v), (mr, vr) in zip(got3, ref3):
        assert torch.equal(m, mr) and torch.equal(v, vr)
    for p in probs:
        p["scene"].close()


def test_static_batched_solve_rejects_more_problems_than_it_holds(W):
    probs = small_problems(W)[:1]
    many = [dict(probs[0], points=probs[0]["points"][:4].contiguous())] * (W.STATIC_MAX_PROBLEMS + 1)
    with pytest.raises(W.WobError, match="capacity"):
        W.solve_batched(many, no_alloc=True)
    probs[0]["scene"].close()
