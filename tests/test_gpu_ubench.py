"""Peak calibration (ubench): every kind runs and reports a rate in a plausible band
around the chip's published figure (256 compute units at 2.4 GHz), and the copy moves
the bytes it claims to."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def md():
    import paper_2104_06311_amd
    return paper_2104_06311_amd


# kind -> (lowest plausible, highest plausible) rate.  Published or unit-count figures:
# exp 1.97e13/s (8 cycles per wave64), FP32 add 7.9e13/s at 2 cycles per wave64 (the
# vector peak, which needs packed instructions; non-packed adds measure about 2.8
# cycles), FP16/BF16 matrix 2.5e15 flop/s, FP32 matrix 1.57e14 flop/s, HBM 8e12 B/s.
BANDS = {"exp": (4e12, 2.6e13), "add_f32": (8e12, 8.2e13), "mfma_f16": (8e14, 2.8e15),
         "mfma_bf16": (8e14, 2.8e15), "mfma_f32": (4e13, 1.8e14), "exp_add2": (3e12, 2.0e13),
         "tile_mix": (2e12, 2.0e13), "tile_mix4": (1.5e12, 2.0e13),
         "tile_mix1": (2e12, 2.0e13)}


@pytest.mark.parametrize("kind", sorted(BANDS))
def test_compute_rates_are_plausible(kind):
    rate, ms = md().ubench(kind)
    lo, hi = BANDS[kind]
    assert lo <= rate <= hi, (kind, rate)
    assert 0.05 < ms < 200.0, (kind, ms)
    # twice the iterations take about twice as long
    doubled = {"exp": 16384, "add_f32": 16384, "mfma_f16": 8192, "mfma_bf16": 8192, "mfma_f32": 4096,
               "exp_add2": 16384, "tile_mix": 2048, "tile_mix4": 1024, "tile_mix1": 2048}
    rate2, ms2 = md().ubench(kind, work=doubled[kind])
    assert 1.5 < ms2 / ms < 2.6, (kind, ms, ms2)


def test_copy_moves_the_bytes():
    nbytes = 1 << 28
    src = torch.arange(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    rate, ms = md().ubench("copy", nbytes, src, dst)
    assert torch.equal(src, dst)
    assert 1e12 <= rate <= 8.5e12, rate
    # a partial copy touches only its prefix
    dst.zero_()
    md().ubench("copy", 4096, src, dst)
    assert torch.equal(dst[:1024], src[:1024]) and int(dst[1024:].abs().max().item()) == 0
    with pytest.raises(ValueError):
        md().ubench("copy", nbytes * 2, src, dst)


def test_exp_add2_mix_is_slower_than_exp_alone():
    """The mix issues three instructions per step on the same port: it cannot beat the
    exponential alone, and it cannot be slower than the three issued one after another."""
    r_exp = md().ubench("exp")[0]
    r_add = md().ubench("add_f32")[0]
    r_mix = md().ubench("exp_add2")[0]
    assert r_mix < r_exp, (r_mix, r_exp)
    serial = 1.0 / (1.0 / r_exp + 2.0 / r_add)
    assert r_mix > 0.8 * serial, (r_mix, serial)


def test_tile_mix_is_bounded_by_its_parts():
    """The demapper's per-tile mix issues the exp + 2 add work of every pair and the two
    matrix products of every tile: it cannot beat the exp + 2 add mix alone, and it cannot
    be slower than that mix and the products issued one after the other."""
    r_mix = md().ubench("exp_add2")[0]
    r_tile = md().ubench("tile_mix")[0]
    r_mfma = md().ubench("mfma_f16")[0]
    assert r_tile < 1.05 * r_mix, (r_tile, r_mix)
    # per exponential: 2 x 32 x 32 x 16 x 2 flop of products per 1024 exponentials
    flop_per_exp = 2.0 * 2 * 32 * 32 * 16 / 1024
    serial = 1.0 / (1.0 / r_mix + flop_per_exp / r_mfma)
    assert r_tile > 0.7 * serial, (r_tile, serial)


def test_more_k_steps_cost_more():
    """Four K steps per tile issue twice the matrix products of two: the mix cannot get
    faster."""
    r2 = md().ubench("tile_mix")[0]
    r4 = md().ubench("tile_mix4")[0]
    assert r4 < 1.05 * r2, (r4, r2)
