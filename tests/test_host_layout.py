"""Host-side packing helpers of the binding (CPU tensors; no GPU needed):
the pitched packing must put every row on an `align` boundary, keep the
pixels, leave the padding zero and round-trip through unpack_pitched."""
import numpy as np
import pytest
import torch

from paper_1909_00149_amd import uot as G


@pytest.mark.parametrize("align", [1, 4, 16, 64])
def test_pack_pitched_round_trip(align):
    rng = np.random.default_rng(0)
    shapes = [(1, 77), (60, 1), (2, 2), (29, 37), (64, 64), (9, 130)]
    ims = [torch.from_numpy(rng.uniform(0.1, 1, s).astype(np.float32)) for s in shapes]
    flat, nx, ny, pitch, offs = G.pack_pitched(ims, align=align)
    assert nx == [s[1] for s in shapes] and ny == [s[0] for s in shapes]
    for a, pt, o in zip(nx, pitch, offs):
        assert pt >= a and pt % align == 0 and pt - a < align
        assert o % align == 0
    back = G.unpack_pitched(flat, nx, ny, pitch, offs)
    for a, b in zip(ims, back):
        assert torch.equal(a, b)
    used = torch.zeros(flat.numel(), dtype=torch.bool)
    for a, b, pt, o in zip(nx, ny, pitch, offs):
        used[o:o + pt * b].view(b, pt)[:, :a] = True
    assert int(used.sum()) == sum(a * b for a, b in zip(nx, ny))
    assert bool((flat[~used] == 0).all())


def test_pack_pitched_align_one_is_pack():
    ims = [torch.ones(3, 5), torch.full((2, 7), 2.0)]
    flat, nx, ny, pitch, offs = G.pack_pitched(ims, align=1)
    ref, nx2, ny2, offs2 = G.pack(ims)
    assert torch.equal(flat, ref) and pitch == nx and offs == offs2


def test_pack_pitched_rejects_bad_align():
    with pytest.raises(ValueError):
        G.pack_pitched([torch.ones(2, 2)], align=0)
