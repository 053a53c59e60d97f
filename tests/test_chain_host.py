"""Host checks of the cluster chaining that feeds Eq. (8) (Sec. 3.2; Sec. 4:
clusters of 12 images, the last three reused as references): membership by
the rule, the fixed first half of the references, and the cluster scenes of
the two-strip, 60-image flight."""
import numpy as np
import pytest

from synth import aerial as A


def test_paper_flight_membership():
    m = A.chain_membership(60, 12, 3)
    assert [own[0] for own, _, _ in m] == [0, 9, 18, 27, 36, 45, 54]
    assert [len(own) for own, _, _ in m] == [12] * 6 + [6]
    for (own, refs, fixed), (prev, _, _) in zip(m[1:], m):
        assert refs == prev[-3:] and own[:3] == refs
        assert fixed == refs[:1]                      # first half of three: one image
    assert m[0][1] == [] and m[0][2] == []


@pytest.mark.parametrize("n,size,ref", [(1, 12, 3), (12, 12, 3), (13, 12, 3), (40, 8, 2), (25, 5, 0), (30, 12, 4),
                                        (50, 20, 5)])
def test_membership_rule(n, size, ref):
    m = A.chain_membership(n, size, ref)
    seen = []
    for c, (own, refs, fixed) in enumerate(m):
        assert 0 < len(own) <= size
        assert own == sorted(own) and len(set(own)) == len(own)
        if c:
            prev = m[c - 1][0]
            assert refs == prev[len(prev) - ref:] if ref else refs == []
            assert fixed == refs[: len(refs) // 2]
            assert len(own) == size or own[-1] == n - 1          # only the last cluster is short
            assert len(own) > len(refs)                          # every cluster brings a new image
        seen += [k for k in own if k not in refs]
    assert seen == list(range(n))                                # every image enters once, in order


def test_membership_rejects_bad_overlap():
    with pytest.raises(ValueError):
        A.chain_membership(10, 4, 4)


def test_chain_scenes():
    ch = A.make_chain(9, pts_per_image=200)
    fl = ch["flight"]
    strip = fl["truth"]["strip"]
    m = A.chain_membership(fl["n_cams"], 12, 3)
    assert len(ch["clusters"]) == len(m)
    for sc, (own, refs, fixed_refs) in zip(ch["clusters"], m):
        ids = list(sc["cam_ids"])
        assert set(own) <= set(ids)
        nb = [k for k in ids if k not in own]
        assert len(nb) <= 8
        for k in nb:                               # neighbours: previous strip of one of the cluster's images
            assert any(strip[k] == strip[i] - 1 for i in own)
        fixed = {int(k) for k, f in zip(ids, sc["fixed"]) if f}
        assert fixed == set(fixed_refs) | set(nb)
        assert int((sc["fixed"] == 0).sum()) <= A_MAX_FREE
        assert list(sc["refs"]) == refs and list(sc["refs_fixed"]) == fixed_refs
        # points: pool points seen at least twice in the cluster, observed only by its cameras
        cnt = np.bincount(sc["obs_pt"], minlength=sc["n_points"])
        assert cnt.min() >= 2
        assert np.array_equal(sc["X"], fl["X"][sc["point_ids"]])


A_MAX_FREE = 24
