"""Pins for the oracle's contact-Hessian conversion (Sec. 4.3 contact barrier, Eq. "gradient and
hessian of contact barrier"; Sec. 5.2 Alg. "Contact Hessian conversion and assembly").

Checked against what the definitions fix, not against the oracle's own products:
- finite differences of a quadratic contact energy written on the vertex positions, where each
  vertex position is evaluated from the CPs by the oracle's surface evaluation (a different code
  path from the weight matrix): central differences are exact for a quadratic up to rounding,
  so the CP Hessian and gradient must match them to near round-off;
- translation invariance (the synthetic pair energies depend on relative positions only, and
  the weights of every vertex sum to one);
- vertices at the four parameter corners, which interpolate single CPs, pass their blocks
  through unchanged;
- the block pattern against the set of CP pairs reached by the vertex supports."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from oracle import contact_ref as cr


def _setup(n_u=9, n_v=7, n_pairs=60, seed=3, spacing=1):
    ku, kv = syn.open_uniform_knots(n_u, spacing), syn.open_uniform_knots(n_v, spacing)
    _, _, rest = syn.flat_sheet(n_u, n_v, spacing=spacing)
    sh = oracle.Sheet(n_u, n_v, ku, kv, rest, 0, 1e4, 0.3, 1e-3, 0, 0, 0, 1e-3, 0.2)
    uv, tris, grid = syn.contact_mesh(n_u, n_v, spacing=spacing)
    pv, H, g = syn.contact_pairs(uv, tris, grid, n_pairs, seed=seed)
    return sh, uv, pv, H, g


def _energy(sh, uv, pv, H, g, C):
    X = np.array([oracle.surface_point(sh, C, u, v) for u, v in uv])
    E = 0.0
    for c in range(pv.shape[0]):
        x = np.zeros(12)
        for s in range(4):
            if pv[c, s] >= 0:
                x[3 * s:3 * s + 3] = X[pv[c, s]]
        E += 0.5 * x @ H[c] @ x + g[c] @ x
    return E


@pytest.mark.parametrize("spacing", [1, 2])
def test_hessian_and_gradient_by_finite_differences(spacing):
    sh, uv, pv, H, g = _setup(spacing=spacing)
    Hc, gc = cr.contact_to_cp(sh, uv, pv, H, g)
    rng = np.random.default_rng(5)
    n = sh.n_cp
    C0 = np.zeros((n, 3))
    for _ in range(3):
        e = rng.standard_normal((n, 3))
        f = rng.standard_normal((n, 3))
        fd = (_energy(sh, uv, pv, H, g, C0 + e + f) - _energy(sh, uv, pv, H, g, C0 + e - f)
              - _energy(sh, uv, pv, H, g, C0 - e + f) + _energy(sh, uv, pv, H, g, C0 - e - f)) / 4.0
        got = e.reshape(-1) @ (Hc @ f.reshape(-1))
        assert abs(got - fd) < 1e-10 * max(1.0, abs(fd))
        fdg = (_energy(sh, uv, pv, H, g, C0 + e) - _energy(sh, uv, pv, H, g, C0 - e)) / 2.0
        assert abs(np.sum(gc * e) - fdg) < 1e-10 * max(1.0, abs(fdg))


def test_translation_invariance():
    sh, uv, pv, H, g = _setup(n_pairs=120)
    Hc, gc = cr.contact_to_cp(sh, uv, pv, H, g)
    for d in range(3):
        t = np.zeros((sh.n_cp, 3))
        t[:, d] = 1.0
        assert np.abs(Hc @ t.reshape(-1)).max() < 1e-12 * abs(Hc).max()
    assert np.abs(gc.sum(axis=0)).max() < 1e-12 * np.abs(gc).max()


def test_corner_vertices_pass_blocks_through():
    n_u, n_v = 8, 6
    ku, kv = syn.open_uniform_knots(n_u), syn.open_uniform_knots(n_v)
    _, _, rest = syn.flat_sheet(n_u, n_v)
    sh = oracle.Sheet(n_u, n_v, ku, kv, rest, 0, 1e4, 0.3, 1e-3, 0, 0, 0, 1e-3, 0.2)
    uv = np.array([[0.0, 0.0], [n_u - 2.0, 0.0], [0.0, n_v - 2.0], [n_u - 2.0, n_v - 2.0]])
    corner_cp = [0, n_u - 1, (n_v - 1) * n_u, n_u * n_v - 1]
    rng = np.random.default_rng(1)
    M = rng.standard_normal((12, 12))
    H = (M @ M.T)[None]
    g = rng.standard_normal((1, 12))
    Hc, gc = cr.contact_to_cp(sh, uv, np.array([[0, 1, 2, 3]]), H, g)
    Hd = Hc.toarray()
    for s in range(4):
        for s2 in range(4):
            i, j = corner_cp[s], corner_cp[s2]
            assert np.allclose(Hd[3 * i:3 * i + 3, 3 * j:3 * j + 3], H[0, 3 * s:3 * s + 3, 3 * s2:3 * s2 + 3], rtol=0, atol=1e-14)
        assert np.allclose(gc[corner_cp[s]], g[0, 3 * s:3 * s + 3], rtol=0, atol=1e-14)
    assert abs(Hd).sum() - abs(H).sum() < 1e-9


def test_block_pattern_matches_vertex_supports():
    sh, uv, pv, H, g = _setup(n_pairs=80, seed=9)
    Hc, _ = cr.contact_to_cp(sh, uv, pv, H, g)
    pat = cr.cp_block_pattern(sh, uv, pv)
    coo = Hc.tocoo()
    blocks = {(int(r) // 3, int(c) // 3) for r, c, v in zip(coo.row, coo.col, coo.data) if v != 0.0}
    assert blocks == pat
