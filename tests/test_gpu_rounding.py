"""The 16-bit store conversion of the sweep (lbm_round16 applies it to an
array): round-to-nearest-even matches IEEE conversion bit for bit; stochastic
rounding returns one of the two neighbouring 16-bit values, leaves
representable values alone, is unbiased (mean over many sites within a few
standard errors of the input), and depends only on (site, plane, seed, step)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2206_12412_amd.lbm import round16  # noqa: E402


def to_bits(t):
    return t.cpu().view(torch.int16).numpy().astype(np.int64) & 0xFFFF


def bf16_rne_bits(x):
    b = x.view(np.uint32).astype(np.uint64)
    return ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) & 0xFFFF


def neighbours(x, fmt):
    """(lower, upper) 16-bit neighbours of each float32 x, as float64."""
    if fmt == "f16s":
        y = x.astype(np.float16)
        with np.errstate(over="ignore"):  # nextafter of the largest FP16 value is inf
            up = np.where(y.astype(np.float32) >= x, y, np.nextafter(y, np.float16(np.inf)))
            lo = np.where(y.astype(np.float32) <= x, y, np.nextafter(y, np.float16(-np.inf)))
        return lo.astype(np.float64), up.astype(np.float64)
    b = x.view(np.uint32)
    t = (b & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)   # towards zero
    away = ((b & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32).astype(np.float64)
    exact = (b & np.uint32(0xFFFF)) == 0
    away = np.where(exact, t, away)
    return np.minimum(t, away), np.maximum(t, away)


def sample(n=1 << 16, seed=0):
    rng = np.random.default_rng(seed)
    mags = 10.0 ** rng.uniform(-9, 3, n)
    x = (mags * rng.choice([-1.0, 1.0], n)).astype(np.float32)
    x[:8] = [0.0, -0.0, 1.0, 2.0 ** -14, 2.0 ** -24, 3 * 2.0 ** -24, 65504.0, -0.5]
    return x


def dev(x):
    return torch.from_numpy(x).cuda()


def test_nearest_matches_ieee_conversion():
    x = sample()
    f16 = to_bits(round16(dev(x), "f16s", "nearest"))
    np.testing.assert_array_equal(f16, x.astype(np.float16).view(np.uint16).astype(np.int64))
    bf = to_bits(round16(dev(x), "bf16s", "nearest"))
    np.testing.assert_array_equal(bf, bf16_rne_bits(x))


@pytest.mark.parametrize("fmt", ["f16s", "bf16s"])
@pytest.mark.parametrize("plane", [0, 1, 2, 3, 4])
def test_stochastic_results_are_neighbours(fmt, plane):
    x = sample(seed=plane)
    out = round16(dev(x), fmt, "stochastic", plane=plane, seed=9, step=123).cpu().float().numpy()
    lo, up = neighbours(x, fmt)
    out = out.astype(np.float64)
    assert np.all((out == lo) | (out == up))
    exact = lo == up
    np.testing.assert_array_equal(out[exact], lo[exact])
    # both neighbours occur
    inexact = ~exact
    assert (out[inexact] == lo[inexact]).any() and (out[inexact] == up[inexact]).any()


@pytest.mark.parametrize("fmt,value", [
    ("f16s", 1.0 + 0.3 * 2.0 ** -10),        # FP16 normal range
    ("f16s", -3.7e-3),
    ("f16s", 5.3 * 2.0 ** -24),               # FP16 subnormal range
    ("f16s", -0.71 * 2.0 ** -24),
    ("bf16s", 1.0 + 0.77 * 2.0 ** -7),
    ("bf16s", -2.345e-6),
])
@pytest.mark.parametrize("plane", [0, 2, 4])
def test_stochastic_rounding_is_unbiased(fmt, value, plane):
    n = 1 << 21
    x = np.full(n, value, dtype=np.float32)
    xv = float(x[0])
    lo, up = neighbours(x[:1], fmt)
    lo, up = float(lo[0]), float(up[0])
    assert lo < xv < up
    out = round16(dev(x), fmt, "stochastic", plane=plane, seed=1, step=7).cpu().float().numpy()
    p_up = float((out.astype(np.float64) == up).mean())
    p = (xv - lo) / (up - lo)
    sigma = np.sqrt(p * (1 - p) / n)
    # 13 (FP16) or 16 (BF16) random bits: the probability is resolved to
    # 2^-13 or better; 2^-12 leaves room for FP16 subnormals, whose move into
    # the binade [2^-14, 2^-13) rounds at 2^-37
    assert abs(p_up - p) <= 5 * sigma + 2.0 ** -12, (p_up, p, sigma)
    mean = out.astype(np.float64).mean()
    assert abs(mean - xv) <= (up - lo) * (5 * sigma + 2.0 ** -12)


def test_draws_depend_on_seed_and_step_only():
    x = dev(sample(seed=3))
    a = to_bits(round16(x, "f16s", "stochastic", plane=1, seed=5, step=10))
    b = to_bits(round16(x, "f16s", "stochastic", plane=1, seed=5, step=10))
    c = to_bits(round16(x, "f16s", "stochastic", plane=1, seed=5, step=11))
    d = to_bits(round16(x, "f16s", "stochastic", plane=1, seed=6, step=10))
    np.testing.assert_array_equal(a, b)
    assert (a != c).any() and (a != d).any()


@pytest.mark.parametrize("fmt", ["f16s", "bf16s"])
def test_draws_of_the_two_sites_of_a_pair_are_uncorrelated(fmt):
    """Two horizontally adjacent sites share one 32-bit hash (16 bits each):
    their round-up decisions are uncorrelated, and so are those of the same
    site in two planes (chained hashes)."""
    n = 1 << 20
    value = 1.0 + 0.3 * 2.0 ** -10 if fmt == "f16s" else 1.0 + 0.3 * 2.0 ** -7
    x = np.full(n, value, dtype=np.float32)
    up = float(neighbours(x[:1], fmt)[1][0])
    a = round16(dev(x), fmt, "stochastic", plane=0, seed=3, step=5).cpu().float().numpy() == up
    b = round16(dev(x), fmt, "stochastic", plane=1, seed=3, step=5).cpu().float().numpy() == up
    bound = 5.0 / np.sqrt(n // 2)
    assert abs(np.corrcoef(a[0::2], a[1::2])[0, 1]) < bound
    assert abs(np.corrcoef(a, b)[0, 1]) < 5.0 / np.sqrt(n)
