"""The allocation-free fine propagator (mcpr_fine_propagate_static) against
mcpr_fine_propagate, through the C ABI: the same kernels in the same order,
so the final states, the slice-end records and the step trace must be equal
bit for bit.  Two calls in a row share the library's static scratch; the
second is smaller than the first, so it runs over what the first left there.
A call that needs more scratch than the array holds is refused before
anything is launched."""
import numpy as np
import pytest

from paper_2310_11365_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import torch
    from paper_2310_11365_amd import mcpr
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return mcpr


def _run_both(mc, ctx, pr, sizes, slice_index):
    """The same sampled ensembles through both entry points."""
    import torch
    pc = mc.problem_c(pr)
    m = pr.steps_per_slice
    xs = []
    for i, P in enumerate(sizes):
        x = torch.empty(P, dtype=mc.torch_dtype(pr.precision), device="cuda")
        ctx.init_particles([pc], [mc.ensemble(x, i)])
        xs.append(x)
    ys = [x.clone() for x in xs]
    n = len(sizes)
    out = []
    for arr, static in ((xs, False), (ys, True)):
        buf = mc.stats_buffer(n, pr.n_regions)
        tr = torch.empty(n * (m + 1) * 2, dtype=torch.float64, device="cuda")
        ens = [mc.ensemble(x, i, slice_index + i) for i, x in enumerate(arr)]
        if static:
            mc.fine_propagate_static([pc], ens, buf, tr)
        else:
            ctx.fine_propagate([pc], ens, buf, tr)
        torch.cuda.synchronize()
        out.append((mc.stats_to_numpy(buf, n, pr.n_regions), tr.cpu().numpy()))
    for x, y in zip(xs, ys):
        assert torch.equal(x, y)
    (s0, t0), (s1, t1) = out
    assert s0.tobytes() == s1.tobytes()
    assert np.array_equal(t0, t1)
    return s1


@pytest.mark.parametrize("prec", [W.FP32, W.FP64])
def test_static_scratch_equals_context_path_two_calls(mc, prec):
    ctx = mc.Context(0)
    ctx.set_graphs(False)
    pr = W.dz_bimodal(P=1000, N=4, T=0.2, precision=prec).problem
    # first call: several ensembles, one above 256 superchunks (the separate
    # mean-field launch), ragged tails; second call: one small ensemble
    rec = _run_both(mc, ctx, pr, [1_100_003, 70_001, 5], 0)
    assert rec[0]["n"][-1] == 1_100_003 and rec[0]["n"][:-1].sum() == 1_100_003
    rec = _run_both(mc, ctx, pr, [1029], 2)
    assert rec[0]["n"][-1] == 1029
    ctx.close()


def test_static_scratch_trig_and_no_outputs(mc):
    """The trigonometric mean field (two-pass records), and a call with
    neither records nor trace."""
    import torch
    ctx = mc.Context(0)
    pr = W.rotator(P=1000, N=4, T=0.2, precision=W.FP64).problem
    _run_both(mc, ctx, pr, [262_147, 3], 1)
    pc = mc.problem_c(pr)
    x = torch.empty(4099, dtype=torch.float64, device="cuda")
    ctx.init_particles([pc], [mc.ensemble(x)])
    y = x.clone()
    ctx.fine_propagate([pc], [mc.ensemble(x, 0, 3)])
    mc.fine_propagate_static([pc], [mc.ensemble(y, 0, 3)])
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    ctx.close()


def test_static_scratch_refuses_oversize_and_unsupported(mc):
    """A call needing more than the static scratch holds is refused with
    MCPR_E_INVALID_ARG (the ensemble is left untouched); the empirical-CDF
    drift is MCPR_E_UNSUPPORTED."""
    import torch
    pr = W.ou_linear(P=1000, N=2, T=0.1, precision=W.FP32).problem
    pc = mc.problem_c(pr)
    P = 150_000_000
    x = torch.zeros(P, dtype=torch.float32, device="cuda")
    buf = mc.stats_buffer(1, 1)
    with pytest.raises(mc.MCPRError) as e:
        mc.fine_propagate_static([pc], [mc.ensemble(x)], buf)
    assert e.value.status == -1 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(x)) == 0
    del x
    pb = W.burgers(P=1000, N=2, T=0.1).problem
    y = torch.zeros(1000, dtype=torch.float64, device="cuda")
    with pytest.raises(mc.MCPRError) as e:
        mc.fine_propagate_static([mc.problem_c(pb)], [mc.ensemble(y)])
    assert e.value.status == -5
