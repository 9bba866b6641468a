import numpy as np

from helpers import round_bf16


def test_round_bf16_known_values():
    # 1 + 2^-8 is the midpoint between 1 and 1 + 2^-7: ties go to even (1.0)
    assert round_bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert round_bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6   # tie, odd -> up
    assert round_bf16(np.array([1.0 + 2.0 ** -8 + 2.0 ** -30]))[0] == 1.0 + 2.0 ** -7
    assert round_bf16(np.array([-0.5]))[0] == -0.5
    assert round_bf16(np.array([0.0]))[0] == 0.0
    x = np.random.default_rng(0).uniform(1e-3, 2.0, 10000)
    r = round_bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))
    # representable: at most 8 significant bits
    m, e = np.frexp(r)
    assert np.all(m * 256 == np.round(m * 256))
