"""The entry point that allocates nothing (lcp_compress_static) against
lcp_compress on a plan with the same parameters, through the C ABI: two calls
in a row, the second with a smaller input, each giving the same records and
permutations as the plan (and the oracle's records), and a request whose
scratch would not fit the static array refused before any work."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_2411_00761_amd import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lcp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_00761_amd import lcp as L
    L.lib()
    return L


def frames_of(sizes, seed):
    rng = np.random.default_rng(seed)
    xs = []
    for j, n in enumerate(sizes):
        if j % 2 == 0:
            xs.append(datagen.uniform_frame(n, hi=100.0, seed=seed + j))
        else:
            xs.append(datagen.clustered_positions(rng, n, 100.0, 30, 0.3))
    return xs


def check_call(lcp, xs, k, max_particles, max_batch_frames):
    xd = [torch.from_numpy(x).cuda() for x in xs]
    out, offs, perms = lcp.compress_static(xd, 1e-4, lcp.EB_REL_GLOBAL, block_log2=k,
                                           max_particles=max_particles,
                                           max_batch_frames=max_batch_frames, want_perm=True)
    plan = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, block_log2=k, max_particles=max_particles,
                    max_batch_frames=max_batch_frames)
    pout, poffs, _, pperms = plan.compress(xd, want_perm=True)
    torch.cuda.synchronize()
    assert offs == poffs
    assert torch.equal(out[:offs[-1]], pout[:poffs[-1]])
    buf = out[:offs[-1]].cpu().numpy().tobytes()
    for j, x in enumerate(xs):
        assert torch.equal(perms[j], pperms[j]), j
        want, wperm, _ = O.compress_s(x, O.grids_for(x, O.EB_REL_GLOBAL, 1e-4), k, 10, j)
        assert buf[offs[j]:offs[j + 1]] == want, j
        assert np.array_equal(perms[j].cpu().numpy().astype(np.uint32), wperm), j


def test_static_scratch_two_calls_second_smaller(lcp):
    # first call: three frames, the largest 400,000 particles, one frame per
    # launch set; second call: two smaller frames, two per launch set
    check_call(lcp, frames_of([400000, 123457, 250001], 5), 6, 400000, 0)
    check_call(lcp, frames_of([70000, 3], 9), 4, 70000, 2)


def test_static_scratch_refuses_what_does_not_fit(lcp):
    x = torch.from_numpy(datagen.uniform_frame(1000, seed=1)).cuda()
    with pytest.raises(lcp.LCPError) as e:
        lcp.compress_static([x], 1e-3, lcp.EB_ABS, block_log2=4, max_particles=1 << 20)
    assert e.value.status == lcp.ERR_BUDGET
    with pytest.raises(lcp.LCPError) as e:
        lcp.compress_static([x], 1e-3, lcp.EB_ABS, block_log2=-1, max_particles=1000)
    assert e.value.status == lcp.ERR_ARG
