"""The device generator reproduces the host generator bit for bit."""
import numpy as np
import pytest

from workloads import configs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("make", [lambda: configs.partitioned(24, 10, 37),
                                  lambda: configs.adi(40, 12, 64),
                                  lambda: configs.poisson(16, 8, 50),
                                  lambda: configs.poisson_complex(16, 8, 50)],
                         ids=["perrow", "smooth", "uniform_d", "uniform_d_complex"])
def test_device_generator_bit_identical(make):
    from workloads import device
    p = make()
    d, coeffs = device.device_inputs(p)
    a, b, c, dh = configs.full_arrays(p)
    assert np.array_equal(d.cpu().numpy(), dh)
    if p.mode == configs.MODE_LIKE_D:
        for t, h in ((coeffs["a"], a), (coeffs["b"], b), (coeffs["c"], c)):
            assert np.array_equal(t.cpu().numpy(), h)


def test_complex_pin_and_extent():
    """The interleaved complex workload spans both right-hand sides and pins
    both parts of mode (0, 0)'s d_0, on the device as on the host."""
    from workloads import device
    p = configs.poisson_complex(8, 4, 12)
    d, _ = device.device_inputs(p)
    assert d.numel() == p.extent() == 2 * 8 * 4 * 12
    assert d[0].item() == 0.0 and d[1].item() == 0.0 and d[2].item() != 0.0
