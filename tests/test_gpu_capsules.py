"""GPU parity of the avatar capsule queries (gs_capsule_queries, through the
C ABI) against the oracle.  Distances are FP32 on the GPU and FP64 in the
oracle: clearances and step gaps must agree within 1e-4 m; the nearest
capsule must attain the clearance (and be the oracle's where the runner-up
is more than 2e-4 m further); the blocked flag must match wherever the
oracle's step gap is further than 1e-4 m from zero (the others are counted
and excluded, a decision taken in a different precision)."""
import sys

import numpy as np
import pytest

from paper_2604_12626_amd import synth

pytestmark = pytest.mark.gpu

F32 = np.float32
TOL = 1e-4
RADIUS, HEIGHT = 0.1, 1.5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2604_12626_amd import binding
    binding.load()
    return torch.device("cuda:0")


def _scene(seed, frames, n_agents, fpos):
    rng = np.random.default_rng(seed)
    clip, first, nfr = synth.avatar_clips(rng, frames)
    caps = synth.capsule_clips(clip)
    now = np.stack([caps[first[a]] for a in range(len(frames))])
    pos, nxt = synth.agents_near_avatars(rng, now, n_agents)
    return caps, first, nfr, np.asarray(fpos, F32), pos, nxt


def _run_gpu(dev, caps, first, nfr, fpos, pos, nxt, aa, with_step=True):
    import torch
    from paper_2604_12626_amd import binding as B
    E = len(pos)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    cl = torch.full((E,), -7.0, device=dev)
    nn = torch.full((E,), -7, dtype=torch.int32, device=dev)
    sg = torch.full((E,), -7.0, device=dev) if with_step else None
    bl = torch.full((E,), 7, dtype=torch.uint8, device=dev) if with_step else None
    B.capsule_queries(t(pos), t(nxt) if with_step else None, t(aa.astype(np.int32)), RADIUS, HEIGHT, t(caps),
                      t(first), t(nfr), t(fpos), cl, nn, sg, bl)
    torch.cuda.synchronize()
    out = [cl.cpu().numpy(), nn.cpu().numpy()]
    if with_step:
        out += [sg.cpu().numpy(), bl.cpu().numpy()]
    return out


def _check(orc, caps, first, nfr, fpos, pos, nxt, aa, got, sample=None):
    idx = np.arange(len(pos)) if sample is None else sample
    n_caps = caps.shape[1]
    cl, nn, sg = orc.capsule_queries(pos[idx], nxt[idx], aa[idx], RADIUS, HEIGHT, caps, first, nfr, fpos, n_caps)
    g_cl, g_nn, g_sg, g_bl = (x[idx] for x in got)
    fin = np.isfinite(cl)
    assert np.array_equal(np.isfinite(g_cl), fin) and np.all(g_nn[~fin] == -1)
    assert np.abs(g_cl[fin] - cl[fin]).max(initial=0.0) <= TOL
    assert np.abs(g_sg[fin] - sg[fin]).max(initial=0.0) <= TOL
    assert np.all(np.isinf(g_sg[~fin]))
    # the GPU's nearest capsule attains the clearance
    for k in np.nonzero(fin)[0]:
        a, c = divmod(int(g_nn[k]), n_caps)
        assert 0 <= a < len(first)
        one, _, _ = orc.capsule_queries(pos[idx[k]:idx[k] + 1], None, np.array([[a, 1]]), RADIUS, HEIGHT,
                                        caps[:, c:c + 1], first, nfr, fpos, 1)
        assert abs(one[0] - cl[k]) <= TOL, (k, one[0], cl[k])
    sure = np.abs(sg) > TOL
    assert np.array_equal(g_bl[sure], (sg[sure] < 0).astype(np.uint8))
    assert set(np.unique(g_bl)) <= {0, 1}
    return int((~sure).sum()), int((sg[sure] < 0).sum())


@pytest.mark.parametrize("fpos", [[0.0, 2.5, 1.25, 7.9], [3.0, -1.0, float("nan"), 100.0]],
                         ids=["fractional", "clamped"])
def test_capsule_queries_parity(dev, orc, fpos):
    caps, first, nfr, fp, pos, nxt = _scene(31, [1, 4, 3, 9], 101, fpos)
    E = len(pos)
    rng = np.random.default_rng(32)
    aa = np.stack([rng.integers(0, 4, E), rng.integers(1, 4, E)], 1)
    aa[::17] = [2, 0]     # no avatars
    aa[5::23] = [-2, 4]   # range clipped to [0, n_avatars)
    nxt[3::11] = pos[3::11]  # zero steps
    say("capsule queries:", E, "agents, fpos", fpos)
    got = _run_gpu(dev, caps, first, nfr, fp, pos, nxt, aa)
    excl, nb = _check(orc, caps, first, nfr, fp, pos, nxt, aa, got)
    say("blocked %d, excluded near zero %d" % (nb, excl))
    assert nb > 0
    zero = np.isfinite(got[0]) & np.all(nxt == pos, 1)
    assert np.allclose(got[2][zero], got[0][zero], atol=TOL)
    # without the step query: same clearances, step outputs untouched
    got2 = _run_gpu(dev, caps, first, nfr, fp, pos, nxt, aa, with_step=False)
    assert np.array_equal(got2[0], got[0]) and np.array_equal(got2[1], got[1])


def test_capsule_queries_full_size(dev, orc):
    # 4099 agents (a ragged last workgroup) around 8 walking avatars of
    # 90-frame clips; the oracle checks a sample of 40 agents
    caps, first, nfr, fp, pos, nxt = _scene(41, [90] * 8, 4099, np.linspace(0.3, 80.7, 8))
    aa = np.tile([0, 8], (len(pos), 1))
    say("capsule queries full size:", len(pos), "agents x", 8 * caps.shape[1], "capsules")
    got = _run_gpu(dev, caps, first, nfr, fp, pos, nxt, aa)
    sample = np.random.default_rng(42).choice(len(pos), 40, replace=False)
    sample = np.union1d(sample, [len(pos) - 1])
    _check(orc, caps, first, nfr, fp, pos, nxt, aa, got, sample=sample)
    assert np.all(np.isfinite(got[0])) and np.all(got[1] >= 0) and np.all(got[2] <= got[0] + TOL)
