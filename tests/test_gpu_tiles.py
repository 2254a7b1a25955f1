"""GPU tests of the MFMA products' tile shapes (tvcs_set_tiles / tvcs_get_tiles and
the autotuner): every shape gives the same bits (no shape changes the order of a
sum), the stats report the shape in use, and shapes that do not exist are refused."""
import sys

import numpy as np
import pytest

from paper_1001_1774_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_1001_1774_amd import tvcs
    tvcs.lib()
    return tvcs


@pytest.fixture(scope="module")
def prob():
    # 48 images: three image tiles, so groups of 32 or more end with a smaller group
    return synth.make_problem("tiles", n=64, m=1229, batch=48, seed_A=71,
                              sigma=[1e-3, 1e-2] * 24, dtype=np.float32)


# {rt, images, kf} of the forward product, then of the adjoint: both k-tile tables,
# both row-tile counts, and group sizes below, at and above the batch
SHAPES = [(2, 16, 4, 2, 16, 4), (4, 16, 4, 4, 16, 4), (2, 32, 4, 4, 32, 2),
          (4, 32, 2, 2, 32, 4), (4, 64, 1, 2, 64, 4), (2, 64, 4, 4, 64, 1),
          (4, 128, 1, 4, 128, 2), (2, 256, 1, 2, 256, 1)]


K = 150   # outer iterations: the first ones are fresh, increments follow


@pytest.mark.parametrize("storage", ["bf16", "bf16_split", "fp8_rowscale"])
def test_every_shape_gives_the_same_bits(T, prob, storage):
    F = prob.f.astype(np.float32)
    with T.Solver(prob.A, prob.n, storage=storage) as s:
        base = s.solve_batch(F, mu=prob.mu, beta=prob.beta, maxit=K, iadm=True)
        auto = s.tiles
        say(f"  {storage}: autotuned shapes {auto}")
        assert all(st["tiles"] == auto for st in base["stats"])
        u0 = base["u"].cpu().numpy()
        it0 = [st["iters"] for st in base["stats"]]
        fr0 = [st["fresh_iters"] for st in base["stats"]]
        assert min(fr0) > 0 and sum(it0) - sum(fr0) > 0   # both product forms ran
        for shape in SHAPES:
            s.tiles = shape
            assert s.tiles == shape
            out = s.solve_batch(F, mu=prob.mu, beta=prob.beta, maxit=K, iadm=True)
            assert out["stats"][0]["tiles"] == shape
            assert [st["iters"] for st in out["stats"]] == it0
            assert [st["fresh_iters"] for st in out["stats"]] == fr0
            same = np.array_equal(out["u"].cpu().numpy(), u0)
            say(f"    shape {shape}: bitwise equal {same}")
            assert same, shape
        s.tiles = None                         # autotune again
        assert s.tiles[1] in (16, 32, 64, 128, 256)


def test_tile_shape_errors(T, prob):
    with T.Solver(prob.A, prob.n, storage="bf16") as s:
        for bad in [(3, 16, 4, 2, 16, 4), (4, 256, 1, 2, 16, 4), (2, 48, 4, 2, 16, 4),
                    (2, 16, 2, 2, 16, 4), (2, 16, 4, 2, 64, 2), (2, 512, 1, 2, 16, 4),
                    (2, 0, 4, 2, 16, 4)]:
            with pytest.raises(T.TvcsError) as ei:
                s.tiles = bad
            assert ei.value.code == T.TVCS_EINVAL, bad
        # the failed calls left the autotuner in charge
        s.solve_batch(prob.f[:3].astype(np.float32), mu=prob.mu, beta=prob.beta, maxit=3,
                      iadm=True)
        assert s.tiles[1] in (16, 32, 64, 128, 256)
        # a forced shape holds across a larger batch's new workspace
        s.tiles = (2, 32, 2, 4, 32, 4)
        out = s.solve_batch(prob.f.astype(np.float32), mu=prob.mu, beta=prob.beta, maxit=3,
                            iadm=True)
        assert out["stats"][0]["tiles"] == (2, 32, 2, 4, 32, 4)
        ms = s.time_products(B=48, reps=2)
        assert ms[0] > 0 and ms[1] > 0
    with T.Solver(prob.A, prob.n, storage="fp32") as s:
        with pytest.raises(T.TvcsError) as ei:
            s.tiles = SHAPES[0]
        assert ei.value.code == T.TVCS_EUNSUPPORTED
        assert s.tiles == (0,) * 6
