"""Pins of the oracle's avatar capsule queries (Sec. 3.3 dynamic NavMesh
blocking with proxy capsules, Sec. 3.4 the clearance and blocked-step query
APIs): the distance routines against brute force over dense samples and
closed forms, and the queries against constructed scenes with known
answers.  CPU only."""
import numpy as np
import pytest

from paper_2604_12626_amd import synth

F32 = np.float32


def _brute_seg_seg(p0, p1, q0, q1, n=401):
    s = np.linspace(0.0, 1.0, n)[:, None]
    P = p0 + s * (p1 - p0)
    Q = q0 + s * (q1 - q0)
    return np.sqrt(((P[:, None, :] - Q[None, :, :]) ** 2).sum(-1)).min()


def test_segment_distance_against_brute_force(orc):
    rng = np.random.default_rng(1)
    for k in range(60):
        p0, p1, q0, q1 = rng.normal(0.0, 1.0, (4, 3))
        if k % 4 == 1:  # parallel pairs
            q1 = q0 + 0.7 * (p1 - p0)
        if k % 4 == 2:  # crossing pairs
            m = p0 + 0.3 * (p1 - p0)
            q1 = 2 * m - q0
        d = orc.segment_segment_distance(p0, p1, q0, q1)
        b = _brute_seg_seg(p0, p1, q0, q1)
        h = (np.linalg.norm(p1 - p0) + np.linalg.norm(q1 - q0)) / 400
        assert d <= b + 1e-12 and b <= d + h, (k, d, b)


def test_segment_distance_closed_forms(orc):
    d = orc.segment_segment_distance
    assert d([0, 0, 0], [1, 0, 0], [0.5, 1, -1], [0.5, 1, 1]) == pytest.approx(1.0, abs=1e-15)  # skew, perpendicular
    assert d([0, 0, 0], [2, 0, 0], [1, 0.5, 0], [3, 0.5, 0]) == pytest.approx(0.5, abs=1e-15)  # parallel overlap
    assert d([0, 0, 0], [1, 0, 0], [3, 0, 0], [5, 0, 0]) == pytest.approx(2.0, abs=1e-15)  # collinear gap
    assert d([0, 0, 0], [1, 1, 0], [1, 0, 0], [0, 1, 0]) == 0.0  # crossing
    assert d([1, 2, 3], [1, 2, 3], [0, 0, 0], [0, 0, 0]) == pytest.approx(np.sqrt(14.0))  # points
    assert d([0, 1, 0], [0, 1, 0], [-1, 0, 0], [1, 0, 0]) == pytest.approx(1.0)
    # symmetric in its two segments and in the orientation of each
    rng = np.random.default_rng(2)
    p0, p1, q0, q1 = rng.normal(0.0, 1.0, (4, 3))
    ref = d(p0, p1, q0, q1)
    for args in ((q0, q1, p0, p1), (p1, p0, q0, q1), (p0, p1, q1, q0)):
        assert d(*args) == pytest.approx(ref, abs=1e-14)


def test_segment_parallelogram_distance_against_brute_force(orc):
    rng = np.random.default_rng(3)
    a = np.linspace(0.0, 1.0, 81)
    for k in range(30):
        s0, s1, o = rng.normal(0.0, 1.0, (3, 3))
        U = rng.normal(0.0, 0.5, 3)
        V = np.array([0.0, 0.0, 1.5])
        if k % 3 == 1:  # a segment through the parallelogram
            c = o + 0.4 * U + 0.6 * V
            s1 = 2 * c - s0
        d = orc.segment_parallelogram_distance(s0, s1, o, U, V)
        S = s0 + np.linspace(0.0, 1.0, 201)[:, None] * (s1 - s0)
        R = (o + a[:, None, None] * U + a[None, :, None] * V).reshape(-1, 3)
        b = np.sqrt(((S[:, None, :] - R[None, :, :]) ** 2).sum(-1)).min()
        h = np.linalg.norm(s1 - s0) / 200 + (np.linalg.norm(U) + np.linalg.norm(V)) / 80
        assert d <= b + 1e-12 and b <= d + h, (k, d, b)
        if k % 3 == 1:
            assert d == 0.0


def test_segment_parallelogram_degenerate_is_a_segment(orc):
    rng = np.random.default_rng(4)
    for _ in range(10):
        s0, s1, o, V = rng.normal(0.0, 1.0, (4, 3))
        assert orc.segment_parallelogram_distance(s0, s1, o, np.zeros(3), V) == pytest.approx(
            orc.segment_segment_distance(s0, s1, o, o + V), abs=1e-14)


def _one_capsule(a, b, r, frames=1):
    caps = np.zeros((frames, 1, 8), F32)
    caps[:, 0, 0:3], caps[:, 0, 3], caps[:, 0, 4:7] = a, r, b
    return caps


def test_capsule_queries_closed_forms(orc):
    # agent (radius 0.1, height 1.5) at the origin; a horizontal capsule of
    # radius 0.05 at height 1 from x = 1 to 2: clearance 1 - 0.15
    caps = _one_capsule([1, 0, 1], [2, 0, 1], 0.05)
    one = (np.array([0], np.int32), np.array([1], np.int32), np.array([0.0], F32))
    pos = np.zeros((3, 3), F32)
    nxt = np.array([[0.5, 0, 0], [-0.5, 0, 0], [0, 3, 0]], F32)  # towards, away, sideways past it
    cl, nn, sg = orc.capsule_queries(pos, nxt, np.tile([0, 1], (3, 1)), 0.1, 1.5, caps, *one, 1)
    assert np.allclose(cl, 0.85, atol=1e-12) and np.all(nn == 0)
    assert sg[0] == pytest.approx(0.35, abs=1e-7) and sg[1] == pytest.approx(0.85, abs=1e-7)
    assert sg[2] == pytest.approx(0.85, abs=1e-7)
    # a capsule above the agent's head: vertical gap
    caps = _one_capsule([-1, 0, 2.0], [1, 0, 2.0], 0.05)
    cl, _, _ = orc.capsule_queries(pos[:1], None, [[0, 1]], 0.1, 1.5, caps, *one, 1)
    assert cl[0] == pytest.approx(0.5 - 0.15, abs=1e-7)
    # a step that passes straight through a thin vertical pole is blocked even
    # though both end positions are clear
    caps = _one_capsule([1, 0, 0], [1, 0, 2], 0.02)
    p = np.array([[0, 0, 0]], F32)
    cl, _, sg = orc.capsule_queries(p, np.array([[2, 0, 0]], F32), [[0, 1]], 0.1, 1.5, caps, *one, 1)
    assert cl[0] == pytest.approx(0.88, abs=1e-7) and sg[0] == pytest.approx(-0.12, abs=1e-7)
    # no avatars: +inf and -1
    cl, nn, sg = orc.capsule_queries(p, p, [[0, 0]], 0.1, 1.5, caps, *one, 1)
    assert cl[0] == np.inf and nn[0] == -1 and sg[0] == np.inf


def test_capsule_queries_interpolate_in_time(orc):
    # the capsule moves from x = 1 to x = 3 over one frame interval: at frame
    # position 0.25 it is at x = 1.5
    caps = np.concatenate([_one_capsule([1, 0, 0], [1, 0, 2], 0.05), _one_capsule([3, 0, 0], [3, 0, 2], 0.05)])
    p = np.zeros((1, 3), F32)
    cl, _, _ = orc.capsule_queries(p, None, [[0, 1]], 0.1, 1.5, caps, np.array([0], np.int32),
                                   np.array([2], np.int32), np.array([0.25], F32), 1)
    assert cl[0] == pytest.approx(1.5 - 0.15, abs=1e-7)


def test_capsule_query_invariants(orc):
    rng = np.random.default_rng(9)
    clip, first, nfr = synth.avatar_clips(rng, [4, 6])
    caps = synth.capsule_clips(clip)
    now = np.stack([caps[first[a]] for a in range(2)])
    pos, nxt = synth.agents_near_avatars(rng, now, 24)
    fpos = np.array([1.5, 3.25], F32)
    aa = np.tile([0, 2], (24, 1))
    cl, nn, sg = orc.capsule_queries(pos, nxt, aa, 0.1, 1.5, caps, first, nfr, fpos, caps.shape[1])
    # the swept step contains the start and the end position
    cl1, _, _ = orc.capsule_queries(nxt, None, aa, 0.1, 1.5, caps, first, nfr, fpos, caps.shape[1])
    assert np.all(sg <= cl + 1e-12) and np.all(sg <= cl1 + 1e-12)
    assert (cl < 0).any() and (cl > 0).any() and (sg < 0).any()
    # a horizontal translation of the whole scene changes nothing
    sh = np.array([0.75, -1.25, 0.0], F32)
    caps2 = caps.copy()
    caps2[..., 0:3] += sh
    caps2[..., 4:7] += sh
    cl2, nn2, sg2 = orc.capsule_queries(pos + sh, nxt + sh, aa, 0.1, 1.5, caps2, first, nfr, fpos, caps.shape[1])
    assert np.allclose(cl2, cl, atol=1e-5) and np.allclose(sg2, sg, atol=1e-5)
    # the nearest capsule attains the clearance
    A = 2
    for e in range(24):
        a, c = divmod(int(nn[e]), caps.shape[1])
        one = caps[:, c:c + 1]
        cle, _, _ = orc.capsule_queries(pos[e:e + 1], None, [[a, 1]], 0.1, 1.5, one, first, nfr, fpos, 1)
        assert cle[0] == pytest.approx(cl[e], abs=1e-12)
