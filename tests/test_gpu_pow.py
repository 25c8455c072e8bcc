"""The power x^y = exp(y log x) that the entropy-carrying kernels share
(entropy p / rho^gamma, rho from the entropy), evaluated on the device
through its probe entry point.  The reference is numpy's FP64 power on the
host, a math-library result rather than the oracle: the point is the
accuracy each form documents, which the FP32-storage parity tests (1e-5)
cannot see.

* library exp and log (FP64-storage kernels): relative error below 1e-14
  for |y log x| < 40;
* short series (FP32-storage kernels): below 5e-14 for x in [e^-12, e^12],
  |y| <= 3 (mostly the truncation of the log series, 2 t^17 / 17 with
  |t| < 0.1716, times |y|);
* zero, negative and non-finite arguments give what exp(y log x) gives in
  IEEE arithmetic, in both forms.
"""
import numpy as np
import pytest
import torch

from gpu_common import require_gpu
from paper_1809_09851_amd import fdbb as F

pytestmark = pytest.mark.gpu

FORMS = [(False, 1e-14), (True, 5e-14)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _device_pow(x: np.ndarray, y: np.ndarray, short: bool) -> np.ndarray:
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    yd = torch.from_numpy(np.ascontiguousarray(y)).cuda()
    out = F.probe_pow(xd, yd, short)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("short, bound", FORMS)
def test_relative_error_over_the_stated_range(short, bound):
    rng = np.random.default_rng(11)
    n = (1 << 20) + 37  # ragged against the 256-thread workgroups
    x = np.exp(rng.uniform(-12.0, 12.0, n))
    y = rng.uniform(-3.0, 3.0, n)
    # the range ends and the exponents the building blocks take:
    # -gamma (entropy) and 1/(gamma - 1) (density from the entropy)
    g = np.array([1.1, 1.3, 1.4, 5.0 / 3.0])
    y[:8] = np.concatenate([-g, 1.0 / (g - 1.0)])
    x[:8] = [np.exp(-12.0), np.exp(12.0), 1.0, 0.5, 2.0, np.sqrt(0.5), np.sqrt(2.0), 1.0 + 2.0 ** -40]
    ref = np.power(x, y)
    got = _device_pow(x, y, short)
    rel = np.abs(got - ref) / ref
    worst = int(np.argmax(rel))
    assert rel[worst] <= bound, (rel[worst], x[worst], y[worst], got[worst], ref[worst])


@pytest.mark.parametrize("short, bound", FORMS)
def test_mantissa_boundaries_and_integers(short, bound):
    """Arguments on both sides of the sqrt(1/2) split of the log's argument
    reduction, powers of two, and integer exponents with exact results."""
    s = np.sqrt(0.5)
    base = np.array([s, np.nextafter(s, 0), np.nextafter(s, 1), 2 * s, np.nextafter(2 * s, 0),
                     np.nextafter(2 * s, 4), 1.0, 2.0, 4.0, 0.25, 1024.0, 2.0 ** -16, 3.0, 10.0])
    x = np.repeat(base, 5)
    y = np.tile(np.array([-3.0, -1.0, 1.0, 2.0, 3.0]), base.size)
    ref = np.power(x, y)
    got = _device_pow(x, y, short)
    assert np.max(np.abs(got - ref) / ref) <= bound


@pytest.mark.parametrize("short", [False, True])
def test_special_values(short):
    tiny = 5e-324  # the smallest subnormal: log is finite, the power overflows
    x = np.array([0.0, 0.0, 0.0, -1.0, -0.0, np.inf, np.inf, np.nan, 1.0, 1e300, 1e-300, tiny, 2.0])
    y = np.array([-1.4, 2.5, 0.0, 1.4, 2.5, -1.4, 2.5, 1.4, np.nan, 2.0, 2.0, -1.4, np.inf])
    with np.errstate(all="ignore"):
        want = np.exp(y * np.log(x))
    got = _device_pow(x, y, short)
    np.testing.assert_array_equal(got, want)


def test_forms_agree_on_the_building_blocks_exponents():
    """On the states the building blocks see (rho and the entropy's base in
    [1e-3, 1e3]), the two forms agree far below the FP32 rounding."""
    rng = np.random.default_rng(12)
    n = 100_003
    x = 10.0 ** rng.uniform(-3.0, 3.0, n)
    y = np.where(rng.random(n) < 0.5, -1.4, 2.5)
    a = _device_pow(x, y, False)
    b = _device_pow(x, y, True)
    assert np.max(np.abs(a - b) / np.abs(a)) <= 6e-14
