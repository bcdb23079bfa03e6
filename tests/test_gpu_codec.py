"""The indexed-map codec on the GPU against the oracle: the index table and
the packed stream bit for bit, and exact round trips."""
import numpy as np
import pytest

import oracle
from paper_1406_0559_amd import inputs
from paper_1406_0559_amd import raylens as rl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = rl.Context(0)
    yield c
    c.close()


def spec_of(p1, p2):
    return inputs.MapSpec(name="codec", kappa=0.5, gamma=0.2, s=0.0, n1=10, n2=10, h1=1.0, h2=1.0,
                          p1=p1, p2=p2, W1=1.0, W2=1.0)


def roundtrip(ctx, c, spec):
    dc = torch.from_numpy(np.ascontiguousarray(c, np.int32)).cuda()
    values, bits, packed = ctx.encode(dc, spec)
    ov, ob, op = oracle.codec_encode(c)
    assert bits == ob
    assert (values.cpu().numpy() == ov).all()
    assert (packed.cpu().numpy().view(np.uint32) == op).all()
    back = ctx.decode(packed, bits, values, spec)
    assert torch.equal(back, dc)


@pytest.mark.parametrize("hi,shape", [(0, (16, 16)), (1, (33, 17)), (255, (257, 131)),
                                      (70000, (301, 203)), (2 ** 31 - 1, (64, 64)),
                                      (1_000_000, (512, 512)), (5000, (4096, 3))])
def test_random_maps(ctx, hi, shape):
    rng = np.random.default_rng(hi % 1000 + 1)
    c = rng.integers(0, hi, size=shape, endpoint=True).astype(np.int32)
    if hi == 2 ** 31 - 1:
        c = np.minimum(c, 3_000_000)        # keep the value histogram to a few MB
    roundtrip(ctx, c, spec_of(shape[1], shape[0]))


def test_unaligned_maps_take_the_general_kernels(ctx):
    """Counts at a 4-byte offset (not 16-byte aligned) encode and decode with
    the word-by-word and pixel-by-pixel kernels: same stream, same map."""
    p1, p2 = 129, 67            # 8643 pixels: two whole 4096-pixel chunks and a tail when aligned
    rng = np.random.default_rng(9)
    c = rng.integers(0, 900, size=(p2, p1)).astype(np.int32)
    spec = spec_of(p1, p2)
    ov, ob, op = oracle.codec_encode(c)
    big = torch.zeros(p1 * p2 + 1, dtype=torch.int32, device="cuda")
    view = big[1:].view(p2, p1)
    view.copy_(torch.from_numpy(c).cuda())
    assert view.data_ptr() % 16 != 0
    values, bits, packed = ctx.encode(view, spec)
    assert bits == ob and (values.cpu().numpy() == ov).all()
    assert (packed.cpu().numpy().view(np.uint32) == op).all()
    out = torch.full((p1 * p2 + 1,), -7, dtype=torch.int32, device="cuda")
    oview = out[1:].view(p2, p1)
    ctx.decode(packed, bits, values, spec, counts=oview)
    assert torch.equal(oview, view)
    assert int(out[0].item()) == -7


def test_shot_maps(ctx):
    for spec in (inputs.config_small(), inputs.config_gerlumph()):
        f = spec.lenses()
        counts, _ = ctx.shoot(rl.DeviceLenses(f.x1, f.x2, f.m), spec, "fp32c")
        roundtrip(ctx, counts.cpu().numpy(), spec)


def test_negative_counts_are_rejected(ctx):
    spec = spec_of(8, 8)
    c = torch.zeros((8, 8), dtype=torch.int32, device="cuda")
    c[3, 3] = -5
    with pytest.raises(rl.RaylensError):
        ctx.encode(c, spec)
