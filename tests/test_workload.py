"""The seeded generators: splitmix64 against its published test vector, ranges,
determinism and the workload recipes' sizes."""
import numpy as np

import workload as W


def test_splitmix64_reference_vector():
    # splitmix64 seeded with 1234567: first outputs of the published reference
    # implementation (Vigna's splitmix64.c)
    z = W.splitmix64(np.uint64(1234567), 5)
    assert [int(v) for v in z] == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                   4593380528125082431, 16408922859458223821]


def test_uniform_ranges_and_determinism():
    a = W.uniform_pm1(1, 2, (4, 5, 6))
    b = W.uniform_pm1(1, 2, (4, 5, 6))
    c = W.uniform_pm1(1, 3, (4, 5, 6))
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, c)
    assert a.min() >= -1 and a.max() < 1 and a.shape == (4, 5, 6)
    r = W.uniform01(9, 0, (100000,))
    assert abs(r.mean() - 0.5) < 0.01


def test_bboxset_recipe():
    d = W.bboxset()
    boxes = d["boxes"]
    assert len(boxes) == 60 and d["ghost"] == 3
    for lev in range(3):
        bl = [b for b in boxes if b["level"] == lev]
        assert len(bl) == 20
        for i, b in enumerate(bl):
            assert all(16 <= v <= 96 for v in b["n"])
            for c in bl[i + 1:]:
                assert not W._overlap(b["lo"], b["n"], c["lo"], c["n"])
    npts = sum(int(np.prod(b["n"])) for b in boxes)
    assert 8e6 < npts < 25e6
    assert d["dt"] == 0.25 / 128


def test_mixed_and_adjoint_recipes_small():
    d = W.mixed_fields(n=16, nfield=2)
    assert len(d["fields"]) == 2 and d["fields"][0].shape == (16, 16, 16)
    np.testing.assert_array_equal(d["A"], d["A"].T)
    for a, kap, phi in d["modes"]:
        assert np.all(np.abs(kap) <= 4) and np.all(np.any(kap != 0, axis=1))
    e = W.adjoint_case(n=16, nsteps=4, checkpoint=2)
    assert 0.5 - 1e-12 <= e["c2"].min() and e["c2"].max() <= 1.5 + 1e-12
