"""The streaming reference kernels behind the HBM rates the fused passes are
compared with (rbicgstab_time_stream through the C ABI): the copy reproduces
its source exactly, the seven-read / three-write mix writes the sums its
definition gives at the stream offsets, the read kernel's per-thread sums add
up to the array's sum, and bad arguments are rejected."""
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


N = (1 << 20) + 777   # not a multiple of the slice or the stream block


def _arrays(torch_mod, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(N)
    return a, torch_mod.as_tensor(a, device="cuda"), torch_mod.zeros(N, dtype=torch_mod.float64, device="cuda")


def test_stream_copy_and_read(rb, torch_mod):
    print("stream copy/read", flush=True)
    a, ad, bd = _arrays(torch_mod, 1)
    ms, by = rb.rbicgstab_time_stream(1, ad, bd, 1024, 3)
    assert ms > 0 and by == 16.0 * N
    assert np.array_equal(bd.cpu().numpy(), a)
    bd.zero_()
    ms, by = rb.rbicgstab_time_stream(0, ad, bd, 512, 3)
    got = bd[: 512 * 256].sum().item()
    assert abs(got - a.sum()) <= 1e-12 * np.abs(a).sum()
    assert np.all(bd[512 * 256:].cpu().numpy() == 0.0)


def test_stream_mix_values(rb, torch_mod):
    print("stream mix", flush=True)
    a, ad, bd = _arrays(torch_mod, 2)
    ms, by = rb.rbicgstab_time_stream(2, ad, bd, 1024, 2)
    length = N // 8 // 1024 * 1024
    ld = length + 512
    assert by == 80.0 * length
    b = bd.cpu().numpy()
    r = np.arange(length)
    v = [a[r + j * ld] for j in range(7)]
    s = ((v[0] + v[1]) + v[2]) + v[3]
    t = (v[4] + v[5]) + v[6]
    assert np.array_equal(b[r], s)
    assert np.array_equal(b[r + ld], t)
    assert np.array_equal(b[r + 2 * ld], s - t)
    assert np.all(b[3 * ld:] == 0.0)


def test_stream_bad_arguments(rb, torch_mod):
    _, ad, bd = _arrays(torch_mod, 3)
    for kind, grid in ((3, 1024), (0, 1004), (1, 0), (0, 8192)):   # 8192 x 256 > N
        with pytest.raises(rb.RbsError):
            rb.rbicgstab_time_stream(kind, ad, bd, grid, 1)
