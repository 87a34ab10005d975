"""The synthetic input generators (CPU): the large-grid mixture generator
against the plain one, and the batched workload's shapes and budgets."""
import numpy as np

from synth import fields as S


def test_torch_mixture_equals_numpy_mixture():
    p = S.random_params(30, (20, 18, 16), seed=3)
    a = S.mixture_field(p, (16, 18, 20), noise=0.0)
    b = S.mixture_field_torch(p, (16, 18, 20)).double().numpy()
    assert np.max(np.abs(a - b)) < 1e-6 * max(1.0, np.max(np.abs(a)))


def test_batch_shapes_respect_the_allowed_dims_and_cap():
    sh = S.batch_shapes(32, seed=11)
    assert len(sh) == 32
    for s in sh:
        assert all(d in S.BATCH_DIMS for d in s)
        assert np.prod(s) <= S.BATCH_MAX_VOXELS
    assert len(set(sh)) > 16                       # uneven
    assert sh == S.batch_shapes(32, seed=11)       # seeded


def test_batch_budgets_follow_energy_within_bounds():
    b = S.batch_budgets([1.0, 2.0, 10.0, 100.0, 0.001])
    assert b[3] == 200000 and b[4] == 8000
    assert b[0] <= b[1] <= b[2] <= b[3]
    assert all(8000 <= v <= 200000 for v in b)


def test_batch_item_fields_are_normalised_and_alternate():
    f0 = S.batch_item_field((24, 20, 16), 0)
    f1 = S.batch_item_field((24, 20, 16), 1)
    for f in (f0, f1):
        assert f.shape == (24, 20, 16)
        assert abs(float(f.min())) < 1e-6 and abs(float(f.max()) - 1.0) < 1e-6
    assert S.gradient_energy(f0) > 0 and S.gradient_energy(f1) > 0
