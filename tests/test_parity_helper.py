"""The comparison the GPU parity tests use (tests/parity.py) catches what a relative L2 norm
alone dilutes: an error confined to one boundary face."""
import numpy as np

from parity import rel, rel_l2, rel_max


def test_face_confined_error_is_caught():
    n = 128
    rng = np.random.default_rng(0)
    ref = 1.0 + 0.1 * rng.standard_normal((n,) * 3)
    got = ref.copy()
    got[:, :, 0] += 5e-10 * np.abs(ref).max()    # one face off by 5e-10 of the field's size
    assert rel_l2(got, ref) < 1e-10               # passes a 1e-10 bound on the norm ...
    assert rel_max(got, ref) >= 5e-10 * (1 - 1e-9)
    assert rel(got, ref) > 1e-10                  # ... but not the combined bound


def test_sequences_compare_pairwise():
    a = [np.ones((2, 2, 2)), np.zeros((3, 3, 3))]
    b = [np.ones((2, 2, 2)), np.zeros((3, 3, 3))]
    assert rel(a, b) == 0.0
    b2 = [np.ones((2, 2, 2)) * 2, np.zeros((3, 3, 3))]
    assert abs(rel_max(a, b2) - 0.5) < 1e-15
    assert abs(rel_l2(a, b2) - 0.5) < 1e-15
