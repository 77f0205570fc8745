"""Host-side helpers of the refined peak search (no GPU): the local lattices
and the far-field angle convention r = -(sin t cos p, sin t sin p, cos t)."""
import numpy as np
import pytest

from paper_2012_09499_amd import refine as RF
import workloads as WL


@pytest.mark.parametrize("radius,dims", [(1, 3), (2, 3), (1, 2), (3, 2)])
def test_lattice_counts_contains_centre_and_is_symmetric(radius, dims):
    L = RF._lattice(radius, dims)
    assert L.shape == ((2 * radius + 1) ** dims, dims)
    assert np.any(np.all(L == 0.0, axis=1))                 # the centre
    assert len({tuple(r) for r in L}) == L.shape[0]          # no duplicates
    assert np.allclose(np.sort(L, axis=0), np.sort(-L, axis=0))
    assert L.min() == -radius and L.max() == radius


def test_direction_and_angles_invert_each_other():
    rng = np.random.default_rng(3)
    t = rng.uniform(0.05, np.pi - 0.05, 200)
    p = rng.uniform(-np.pi + 0.05, np.pi - 0.05, 200)
    d = RF._direction(t, p)
    np.testing.assert_allclose(np.linalg.norm(d, axis=-1), 1.0, rtol=0, atol=1e-15)
    t2, p2 = RF._angles(d)
    np.testing.assert_allclose(t2, t, rtol=0, atol=1e-12)
    np.testing.assert_allclose(p2, p, rtol=0, atol=1e-12)


def test_direction_matches_the_candidate_grid_convention():
    # the half-sphere candidate grid of the far-field workloads uses the same
    # convention, so refining from a grid direction starts exactly on it
    d = WL.half_sphere_directions(10.0)
    t, p = RF._angles(d)
    np.testing.assert_allclose(RF._direction(t, p), d, rtol=0, atol=1e-12)


def test_far_field_spacing_is_radians():
    assert RF.grid_spacing_far(2.0) == pytest.approx(np.pi / 90.0)
