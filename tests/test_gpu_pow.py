"""The power x^y = exp(y log x) that the entropy-carrying kernels share
(entropy p / rho^gamma, rho from the entropy), evaluated on the device
through its probe entry point.  The reference is numpy's FP64 power on the
host, a math-library result rather than the oracle: the point is the
accuracy each form documents, which the FP32-storage parity tests (1e-5)
cannot see.

* library exp and log (FP64-storage kernels): relative error below 1e-14
  for |y log x| < 40;
* base-2 form (FP32-storage kernels: FP64 exponent split and scaling,
  hardware FP32 log2 and exp2 of the reduced arguments): below 6e-7 for
  |y| <= 3, from |y| ln 2 (2^-24 / ln 2 + 2^-24) + 2^-24 ln 2 + 2^-23;
* zero, negative and non-finite arguments give what exp(y log x) gives in
  IEEE arithmetic, in both forms.
"""
import numpy as np
import pytest
import torch

from gpu_common import require_gpu
from paper_1809_09851_amd import fdbb as F

pytestmark = pytest.mark.gpu

FP32_FORM_BOUND = 6e-7
FORMS = [(False, 1e-14), (True, FP32_FORM_BOUND)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _device_pow(x: np.ndarray, y: np.ndarray, fp32_form: bool) -> np.ndarray:
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    yd = torch.from_numpy(np.ascontiguousarray(y)).cuda()
    out = F.probe_pow(xd, yd, fp32_form)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("fp32_form, bound", FORMS)
def test_relative_error_over_the_stated_range(fp32_form, bound):
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
    got = _device_pow(x, y, fp32_form)
    rel = np.abs(got - ref) / ref
    worst = int(np.argmax(rel))
    assert rel[worst] <= bound, (rel[worst], x[worst], y[worst], got[worst], ref[worst])


@pytest.mark.parametrize("fp32_form, bound", FORMS)
def test_mantissa_boundaries_and_integers(fp32_form, bound):
    """Arguments at and next to powers of two (the ends of the mantissa
    range of the base-2 decomposition) and integer exponents."""
    s = np.sqrt(0.5)
    base = np.array([s, np.nextafter(s, 0), np.nextafter(s, 1), 2 * s, 0.5, np.nextafter(0.5, 0),
                     np.nextafter(0.5, 1), np.nextafter(1.0, 0), 1.0, 2.0, 4.0, 0.25, 1024.0, 2.0 ** -16,
                     3.0, 10.0])
    x = np.repeat(base, 5)
    y = np.tile(np.array([-3.0, -1.0, 1.0, 2.0, 3.0]), base.size)
    ref = np.power(x, y)
    got = _device_pow(x, y, fp32_form)
    assert np.max(np.abs(got - ref) / ref) <= bound
    if fp32_form:
        # powers of two to integer exponents are exact in the base-2 form
        # (log2 of the mantissa 1/2 and 2^0 are exact); exp(y log x) of the
        # FP64 form only meets its relative bound there
        two = np.array([0.5, 2.0, 4.0, 0.25, 1024.0, 2.0 ** -16])
        xi = np.repeat(two, 4)
        yi = np.tile(np.array([-3.0, -1.0, 2.0, 3.0]), two.size)
        np.testing.assert_array_equal(_device_pow(xi, yi, True), np.power(xi, yi))


@pytest.mark.parametrize("fp32_form", [False, True])
def test_special_values(fp32_form):
    tiny = 5e-324  # the smallest subnormal: log is finite, the power overflows
    x = np.array([0.0, 0.0, 0.0, -1.0, -0.0, np.inf, np.inf, np.nan, 1.0, 1e300, 1e-300, tiny, 2.0])
    y = np.array([-1.4, 2.5, 0.0, 1.4, 2.5, -1.4, 2.5, 1.4, np.nan, 2.0, 2.0, -1.4, np.inf])
    with np.errstate(all="ignore"):
        want = np.exp(y * np.log(x))
    got = _device_pow(x, y, fp32_form)
    np.testing.assert_array_equal(got, want)


def test_fp32_form_on_the_building_blocks_arguments():
    """On the states the building blocks see (rho and the entropy's base in
    [1e-3, 1e3], y = -gamma or 1/(gamma-1)) the FP32-storage form stays
    within its bound of the FP64 form, and after rounding to FP32 within a
    few units in the last place of the correctly rounded power."""
    rng = np.random.default_rng(12)
    n = 100_003
    x = 10.0 ** rng.uniform(-3.0, 3.0, n)
    y = np.where(rng.random(n) < 0.5, -1.4, 2.5)
    a = _device_pow(x, y, False)
    b = _device_pow(x, y, True)
    assert np.max(np.abs(a - b) / np.abs(a)) <= FP32_FORM_BOUND
    a32, b32 = a.astype(np.float32), b.astype(np.float32)
    ulps = np.abs(a32.view(np.int32).astype(np.int64) - b32.view(np.int32).astype(np.int64))
    assert ulps.max() <= 12
