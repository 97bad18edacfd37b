"""Pins of the oracle's neighbour search (Sec. 3.2, App. B) against brute force and lattice counts."""
import numpy as np
import pytest

from paper_2507_21684_amd.inputs import SimSpec, make_state


def _lattice_count(dim, R):
    """Integer lattice points strictly inside radius R (closed-form count by enumeration)."""
    r = np.arange(-R, R + 1)
    g = np.array(np.meshgrid(*[r] * dim, indexing="ij")).reshape(dim, -1)
    return int(np.sum((g ** 2).sum(0) < R * R))


@pytest.mark.parametrize("dim,side", [(2, 32), (3, 16)])  # dyadic dx: r = H is exact
def test_perfect_lattice_counts(orc, dim, side):
    spec = SimSpec(dim, side, jitter=0.0)
    x, _, _ = make_state(spec, 0)
    for prec in ("f64", "f32"):
        off, idx = orc.neighbors(x, 1.0, spec.H, prec)
        counts = np.diff(off)
        assert np.all(counts == _lattice_count(dim, 4)), np.unique(counts)
    assert _lattice_count(2, 4) == 45 and _lattice_count(3, 4) == 251


def _brute_numpy(x, L, H):
    """Independent O(N^2) reference in float64: minimum image by rounding, strict r < H.
    Returns the set of pairs and the set of pairs whose r^2 is within 1e-9 H^2 of H^2."""
    dim, n = x.shape
    u = x - L * np.floor(x / L)
    d = u[:, :, None] - u[:, None, :]
    d = d - L * np.round(d / L)
    r2 = (d ** 2).sum(0)
    inside = r2 < H * H
    near = np.abs(r2 - H * H) < 1e-9 * H * H
    return inside, near


@pytest.mark.parametrize("dim,side,seed", [(2, 16, 0), (2, 20, 1), (3, 10, 2), (3, 13, 3)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_grid_matches_brute_force(orc, dim, side, seed, prec):
    spec = SimSpec(dim, side, jitter=0.45)
    x, _, _ = make_state(spec, seed)
    # unwrapped positions: shift some particles by whole boxes
    rng = np.random.default_rng(seed)
    x = x + rng.integers(-2, 3, size=x.shape).astype(np.float64)
    if prec == "f32":
        x = x.astype(np.float32).astype(np.float64)
    off_g, idx_g = orc.neighbors(x, 1.0, spec.H, prec, brute=False)
    off_b, idx_b = orc.neighbors(x, 1.0, spec.H, prec, brute=True)
    np.testing.assert_array_equal(off_g, off_b)
    np.testing.assert_array_equal(idx_g, idx_b)
    inside, near = _brute_numpy(x, 1.0, spec.H)
    n = x.shape[1]
    for i in range(n):
        row = idx_g[off_g[i]:off_g[i + 1]]
        assert np.all(np.diff(row) > 0), "rows ascending, no duplicates"
        assert i in row, "self included"
        ref = np.nonzero(inside[i])[0]
        amb = set(np.nonzero(near[i])[0].tolist())
        assert set(row.tolist()) ^ set(ref.tolist()) <= amb


def test_relation_is_symmetric(orc):
    spec = SimSpec(3, 12, jitter=0.3)
    x, _, _ = make_state(spec, 9)
    off, idx = orc.neighbors(x, 1.0, spec.H, "f32")
    pairs = set()
    for i in range(x.shape[1]):
        for j in idx[off[i]:off[i + 1]]:
            pairs.add((i, int(j)))
    assert all((j, i) in pairs for (i, j) in pairs)


def test_rejects_support_too_large(orc):
    x = np.zeros((2, 4))
    with pytest.raises(ValueError):
        orc.neighbors(x, 1.0, 0.5)


def test_empty(orc):
    off, idx = orc.neighbors(np.zeros((2, 0)), 1.0, 0.1)
    assert off.tolist() == [0] and idx.size == 0
