"""The multigrid cycle's kernel forms (ccns_params.mg_forms, chosen per level
by the tuner) compute the same values bit for bit: pressure solves and a
step with every level in each of the five forms (the finest level's
up-sweep, whose tiles fix the order of the statistics' sums, in the tall
ones) equal the defaults' exactly, in FP64 and in precision 1, on a grid
whose hierarchy has levels of both default forms (tall and short tiles)."""

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import case_setup

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("precision", [0, 1])
def test_forms_agree_bit_for_bit(precision):
    from paper_2211_10698_amd import ccns, tune
    case = W.scaled_cylinder(1030, 517, 10.3, 5.17, seed=4)
    caps, pr, st, ctx, Dx, Dy = case_setup(case, pcg_tol=1e-10, precision=precision)
    levels = ctx.mg_levels()
    print(f"[mg-forms] levels {levels}", flush=True)
    assert len(levels) >= 3
    kinds = {(d, u) for _, _, d, u in levels}
    assert len(kinds) >= 2      # the defaults differ between levels
    rng = np.random.default_rng(8)
    b = torch.from_numpy(np.where(pr.act_p, rng.uniform(-1, 1, pr.act_p.shape), 0.0)).cuda()
    zero = torch.zeros_like(b)

    def solve(word):
        ctx.set_mg_forms(word)
        ctx.set_field(ccns.F_PHI, zero)
        phi, info, status = ctx.pressure_solve(b)
        assert status == 0
        return phi.cpu().numpy(), info.iterations

    ref, it_ref = solve(0)
    for f in (1, 2, 3, 4, 5):
        # the finest level's up-sweep keeps tall tiles (its statistics' order)
        pairs = [(f, f if f <= 3 else 2)] + [(f, f)] * (len(levels) - 1)
        word = tune.pack(pairs)
        ctx.set_mg_forms(word)
        assert [(d, u) for _, _, d, u in ctx.mg_levels()] == pairs
        phi, it = solve(word)
        assert it == it_ref and np.array_equal(phi, ref), f
    # one step from the same state with mixed forms
    s0 = W.perturbation(case)
    ux0 = np.where(pr.act_u, case.u_inf + s0[0], Dx)
    uy0 = np.where(pr.act_v, s0[1], Dy)
    out = []
    for word in (0, tune.pack([(2, 1), (4, 3)] + [(3, 2)] * (len(levels) - 2))):
        ctx.set_mg_forms(word)
        for f, v in ((ccns.F_UX, ux0), (ccns.F_UY, uy0), (ccns.F_P, np.zeros_like(ux0)),
                     (ccns.F_PHI, np.zeros_like(ux0))):
            ctx.set_field(f, v)
        ctx.project()
        ctx.step(1)
        out.append([ctx.get_field(f).cpu().numpy() for f in (ccns.F_UX, ccns.F_UY, ccns.F_P)])
    for a, c in zip(*out):
        assert np.array_equal(a, c)
    with pytest.raises(ccns.CcnsError):
        ctx.set_mg_forms(7)
    with pytest.raises(ccns.CcnsError):
        ctx.set_mg_forms(4 << 3)
    with pytest.raises(ccns.CcnsError):
        ctx.set_mg_forms(5 << 3)
    with pytest.raises(ccns.CcnsError):
        ctx.set_mg_forms(6)
    ctx.close()


def test_cached_forms_apply():
    """The committed cache is keyed by this GPU's architecture and gives a
    512 x 512 context its tuned forms."""
    from paper_2211_10698_amd import tune
    cache = tune.load_cache()
    dev = tune.device_key()
    print(f"[mg-forms] device {dev}", flush=True)
    assert dev in cache
    g = W.GridSpec(512, 512, 0.0, 0.0, 1.0, 1.0)
    case = W.Case("forms_512", g, [W.Body(W.CIRCLE, 0.5, 0.5, a=0.15)], re=100.0)
    from paper_2211_10698_amd import ccns
    caps = ccns.ccns_capacities_device(g, case.bodies).cpu().numpy()
    Dx, Dy = W.dirichlet(case)
    ctx = ccns.Context(g, ccns.make_params(1.0, case.mu, case.tau), caps, Dx, Dy)
    word = tune.apply_cached(ctx, 0)
    assert word != 0
    got = [(d, u) for _, _, d, u in ctx.mg_levels()]
    assert got[0] == tuple(cache[dev]["f64"]["512x512"])
    ctx.close()
