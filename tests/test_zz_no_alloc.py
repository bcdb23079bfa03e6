"""rl_shoot_noalloc, the shoot entry point for callers that cannot allocate,
against rl_shoot: the same counts and escaped count bit for bit, on two calls
in a row (the second with a smaller lens field and ray grid, so it runs over
what the first left in the shared staging array), in both precisions; and
its lens-count limit refused on the host."""
import dataclasses

import numpy as np
import pytest

from paper_1406_0559_amd import inputs
from paper_1406_0559_amd import raylens as rl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a HIP device")
    c = rl.Context(0)
    yield c
    c.close()


def _calls():
    base = inputs.config_small()
    # 5000 mass-weighted lenses (20 compensation blocks minus a ragged tail)
    # on a ragged 700 x 515 grid, then 333 unit lenses on 300 x 261
    first = dataclasses.replace(base, name="noalloc-first", n1=700, n2=515, n_lens=5000,
                                disc_radius=(5000 / 0.4) ** 0.5, masses="salpeter", seed=11)
    second = dataclasses.replace(base, name="noalloc-second", n1=300, n2=261, p1=200, p2=180,
                                 n_lens=333, disc_radius=(333 / 0.4) ** 0.5, masses="unit",
                                 seed=12)
    return first, second


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_noalloc_equals_rl_shoot_on_two_calls(ctx, prec):
    import torch
    for spec in _calls():
        print(f"  rl_shoot_noalloc {prec} {spec.name}: {spec.n1}x{spec.n2} rays, "
              f"{spec.n_lens} lenses", flush=True)
        f = spec.lenses()
        L = rl.DeviceLenses(f.x1, f.x2, f.m)
        want_c, want_e = ctx.shoot(L, spec, prec)
        got_c, got_e = ctx.new_map(spec)
        ctx.shoot_noalloc(L, spec, prec, got_c, got_e)
        torch.cuda.synchronize()
        assert int(got_c.sum().item()) + int(got_e.item()) == spec.rays
        assert torch.equal(got_c, want_c)
        assert int(got_e.item()) == int(want_e.item())


def test_noalloc_row_ranges_add_up(ctx):
    """Two row ranges through the no-allocation entry equal one whole map."""
    import torch
    spec = _calls()[0]
    f = spec.lenses()
    L = rl.DeviceLenses(f.x1, f.x2, f.m)
    want_c, want_e = ctx.shoot(L, spec, "fp32c")
    got_c, got_e = ctx.new_map(spec)
    ctx.shoot_noalloc(L, spec, "fp32c", got_c, got_e, 0, 200)
    ctx.shoot_noalloc(L, spec, "fp32c", got_c, got_e, 200, spec.n2)
    torch.cuda.synchronize()
    assert torch.equal(got_c, want_c)
    assert int(got_e.item()) == int(want_e.item())


def test_noalloc_refuses_fields_above_its_limit(ctx):
    n = rl.RL_NOALLOC_MAX_LENSES + 1
    spec = dataclasses.replace(_calls()[1], n_lens=n)
    L = rl.DeviceLenses(np.zeros(n), np.zeros(n))
    c, e = ctx.new_map(spec)
    with pytest.raises(rl.RaylensError) as err:
        ctx.shoot_noalloc(L, spec, "fp32c", c, e)
    assert err.value.status == rl.RL_E_INVALID
    assert "at most" in str(err.value)
    assert int(c.abs().sum().item()) == 0 and int(e.item()) == 0
