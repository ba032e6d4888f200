"""Shared helpers for the GPU parity tests (no arithmetic of the method lives here)."""
import numpy as np

import oracle
import synthetic as syn


def oracle_sheet(scene_or_parts, material=None):
    if isinstance(scene_or_parts, syn.Scene):
        sc = scene_or_parts
        m = sc.material
        return oracle.Sheet(sc.n_u, sc.n_v, sc.knots_u, sc.knots_v, sc.rest, m.membrane, m.young, m.poisson,
                            m.thickness, m.mu_st1, m.mu_st2, m.mu_sh, m.mu_bend, m.rho_area)
    n_u, n_v, ku, kv, rest = scene_or_parts
    m = material
    return oracle.Sheet(n_u, n_v, ku, kv, rest, m.membrane, m.young, m.poisson, m.thickness, m.mu_st1, m.mu_st2,
                        m.mu_sh, m.mu_bend, m.rho_area)


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rowwise_err(got, ref, axis=-1, floor=1e-3):
    """Worst entry error of ``got`` against ``ref``, each entry scaled by the largest magnitude
    of its row (the entries that share an index along ``axis``: one element, one CP), the scale
    floored at ``floor`` times the largest magnitude of the whole array.

    A single norm over a whole array (``relerr``) lets an error confined to a few rows pass at
    up to sqrt(rows) times its bound; this bounds every row against its own size."""
    g = np.asarray(got, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    assert g.shape == r.shape, (g.shape, r.shape)
    if g.ndim == 0:
        g, r = g.reshape(1), r.reshape(1)
    ax = axis % g.ndim
    g = np.moveaxis(g, ax, 0).reshape(g.shape[ax], -1)
    r = np.moveaxis(r, ax, 0).reshape(r.shape[ax], -1)
    scale = np.abs(r).max(axis=1)
    scale = np.maximum(scale, floor * max(float(scale.max()), 1e-300))
    return float((np.abs(g - r).max(axis=1) / scale).max())


def upper27(H):
    """(ne, 27, 27) -> (378, ne) upper triangle, row-major over r <= c."""
    iu = np.triu_indices(27)
    return H[:, iu[0], iu[1]].T


def oracle_stencil_to_upper(H, n_u, n_v):
    """Oracle stencil form (n_cp, 25, 3, 3) -> the library's upper-stencil layout (114, n_cp)."""
    from paper_2506_18867_amd.bsc import SLOT_OFFSETS
    n = n_u * n_v
    out = np.zeros((114, n))
    d = H[:, 12]
    out[0], out[1], out[2], out[3], out[4], out[5] = d[:, 0, 0], d[:, 0, 1], d[:, 0, 2], d[:, 1, 1], d[:, 1, 2], d[:, 2, 2]
    for s in range(1, 13):
        di, dj = SLOT_OFFSETS[s]
        slot25 = (dj + 2) * 5 + (di + 2)
        out[6 + 9 * (s - 1): 6 + 9 * s] = H[:, slot25].reshape(n, 9).T
    # blocks that leave the grid are zero on both sides
    a = np.arange(n)
    i, j = a % n_u, a // n_u
    for s in range(1, 13):
        di, dj = SLOT_OFFSETS[s]
        bad = (i + di < 0) | (i + di >= n_u) | (j + dj >= n_v)
        out[6 + 9 * (s - 1): 6 + 9 * s, bad] = 0.0
    return out


def deformed(scene, seed, amp=0.05, noise=0.0):
    x = scene.x0 + syn.smooth_field(scene.n_u, scene.n_v, seed, amp=amp)
    if noise:
        x = x + noise * np.random.default_rng(seed).standard_normal(x.shape)
    return x
