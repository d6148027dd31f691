"""The Ritz step's Gram product X^T Y (library kernels through the C ABI) against
NumPy on the same operands: every tile shape class (interior 128 x 128 tiles,
32-granular right and bottom edges, corner), the symmetric upper-triangle path,
the small-product path, and row counts that are not a multiple of the 16-row
slabs (the last slab of the last row chunk goes through masked loads).

The reference is np.dot in FP64; the bound is a few units of rounding of the
sum of term magnitudes, sqrt(n) eps |X|^T |Y| for random operands."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def rb():
    from paper_1406_2831_amd import rbicgstab as rbm
    rbm.load_library()
    return rbm


def _check(rb, torch_mod, n, mx, my, sym, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((mx, n))
    Y = X if sym else rng.standard_normal((my, n))
    print(f"gram n={n} mx={mx} my={my} sym={sym}", flush=True)
    Xd = torch_mod.as_tensor(X, device="cuda")
    Yd = Xd if sym else torch_mod.as_tensor(Y, device="cuda")
    got = rb.rbicgstab_gram(Xd, Yd).cpu().numpy().T   # mx x my
    ref = X @ Y.T
    mag = np.abs(X) @ np.abs(Y).T
    err = np.abs(got - ref) / mag
    assert got.shape == (mx, my)
    assert err.max() <= 8 * np.sqrt(n) * np.finfo(float).eps, err.max()
    if sym:
        assert np.array_equal(got, got.T)


@pytest.mark.parametrize("n,mx,my,sym", [
    (1681, 186, 186, True),     # one interior tile + edges, tail of 1 row in the last chunk
    (1681, 186, 200, False),
    (20007, 276, 276, True),    # 2 x 2 interior tiles (upper triangle), 32-granular edges
    (20007, 276, 300, False),
    (4099, 128, 128, False),    # interior only
    (4099, 40, 60, False),      # below the matrix-core sizes: the 64-tile kernel
    (262144, 282, 282, True),   # the benchmark's store size
    (20007, 323, 323, True),    # 96-wide edges (the first shift's store size)
    (20007, 323, 250, False),   # 96-wide bottom edge, 128-wide right edge
    (4099, 228, 300, False),    # 128-wide bottom edge (100 valid), 64-wide right edge (44 valid)
])
def test_gram_matches_numpy(rb, torch_mod, n, mx, my, sym):
    _check(rb, torch_mod, n, mx, my, sym, seed=n + mx + my)


def test_gram_rejects_bad_arguments(rb, torch_mod):
    lib = rb.load_library()
    assert lib.rbicgstab_gram_workspace_bytes(0, 4, 4) == 0
    X = torch_mod.zeros((4, 16), dtype=torch_mod.float64, device="cuda")
    rc = lib.rbicgstab_gram(16, rb._ptr(X), 8, 4, rb._ptr(X), 16, 4, rb._ptr(X), None, 0, None)
    assert rc == -1   # ldx < n
