"""xy_label_links_noalloc (the labelling with the library's fixed device
scratch) against xy_label_links (per-call scratch), through the C ABI.

Integer work: the canonical labels must be equal element by element.  Two
calls in a row on one device, the second with a smaller lattice, so that the
second runs over what the first left in the shared scratch; then a size past
the scratch is refused before anything is enqueued.
"""
import numpy as np
import pytest
import torch

from paper_1210_6116_amd import _lib

pytestmark = pytest.mark.gpu


def _links(L, seed, p):
    rng = np.random.default_rng(seed)
    return rng.random(L * L) < p, rng.random(L * L) < p


def _planes(bx, by, N):
    words = max(1, (N + 31) // 32)

    def pack(b):
        bits = np.zeros(words * 32, dtype=np.uint8)
        bits[:N] = b
        return torch.from_numpy(np.packbits(bits, bitorder="little").view(np.int32).copy()).cuda()

    return pack(bx), pack(by)


def _both(L, bits, rows, seed, p):
    N = L * L
    bx, by = _links(L, seed, p)
    dbx, dby = _planes(bx, by, N)
    dt = torch.int64 if bits == 64 else torch.int32
    ref = torch.full((N,), -1, dtype=dt, device="cuda")
    got = torch.full((N,), -1, dtype=dt, device="cuda")
    stream = torch.cuda.current_stream()
    print("no-alloc labelling L=%d bits=%d rows=%d seed=%d p=%.2f" % (L, bits, rows, seed, p), flush=True)
    _lib.xy_label_links(L, bits, rows, dbx.data_ptr(), dby.data_ptr(), ref.data_ptr(), stream.cuda_stream)
    _lib.xy_label_links_noalloc(L, bits, rows, dbx.data_ptr(), dby.data_ptr(), got.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def _check_canonical(lab, L):
    """Every label is a site of its own cluster's minimum: lab[lab[i]] == lab[i] <= i."""
    idx = np.arange(L * L)
    assert np.all(lab <= idx)
    assert np.array_equal(lab[lab], lab)


@pytest.mark.parametrize("first,second", [((512, 32, 0, 0.6), (128, 32, 16, 0.45)),
                                          ((2048, 64, 16, 0.5), (256, 32, 64, 0.55))])
def test_noalloc_matches_label_links_twice(first, second):
    for k, (L, bits, rows, p) in enumerate((first, second)):
        ref, got = _both(L, bits, rows, 1000 + k, p)
        assert np.array_equal(ref, got), "call %d (L=%d) differs at %d sites" % (k, L, int((ref != got).sum()))
        _check_canonical(got.astype(np.int64), L)


def test_noalloc_refuses_sizes_past_its_scratch():
    L = 4096
    d = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(_lib.XYError) as ei:
        _lib.xy_label_links_noalloc(L, 32, 32, d.data_ptr(), d.data_ptr(), d.data_ptr(), None)
    assert ei.value.code == _lib.XY_EINVAL
    assert "scratch" in str(ei.value)
