"""Full-Stokes oracle against facts fixed without it: polarisation states
built from a common signal give the textbook Stokes vectors exactly (linear
at 0, 90 and 45 degrees, circular of both hands), orthogonal X and Y codes
are unpolarised, a fully polarised source satisfies I^2 = Q^2 + U^2 + V^2,
and cross-feed products are taken from the right triangle entries (checked
against products formed directly from the voltages)."""
import numpy as np
import pytest

import oracle
from oracle import stokes as st


def _vis(x):
    """Exact visibilities of complex integer voltages x [N][T] for one
    channel, by the X-engine oracle: [1][P][2]."""
    N, T = x.shape
    v = np.zeros((T, 1, N, 2), np.int8)
    v[..., 0] = x.T.real[:, None, :]
    v[..., 1] = x.T.imag[:, None, :]
    return oracle.xcorr(v.reshape(-1).view(np.int8), 8, T, 1, N)


def _sig(T, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(-20, 21, T) + 1j * rng.integers(-20, 21, T)


def _auto_stokes(x_x, x_y):
    s = st.stokes(_vis(np.stack([x_x, x_y])), 2)[0, 0]
    return s[:, 0] + 1j * s[:, 1]       # I, Q, U, V as complex numbers


def test_textbook_states():
    s = _sig(64, 1)
    P = float(np.sum(np.abs(s) ** 2))
    z = np.zeros_like(s)
    I, Q, U, V = _auto_stokes(s, z)                 # linear, X only
    assert (I, Q, U, V) == (P, P, 0, 0)
    I, Q, U, V = _auto_stokes(z, s)                 # linear, Y only
    assert (I, Q, U, V) == (P, -P, 0, 0)
    I, Q, U, V = _auto_stokes(s, s)                 # linear at 45 degrees
    assert (I, Q, U, V) == (2 * P, 0, 2 * P, 0)
    I, Q, U, V = _auto_stokes(s, -1j * s)           # Y lags X by 90 degrees
    assert (I, Q, U, V) == (2 * P, 0, 0, 2 * P)
    I, Q, U, V = _auto_stokes(s, 1j * s)            # the other hand
    assert (I, Q, U, V) == (2 * P, 0, 0, -2 * P)


def test_orthogonal_codes_are_unpolarised():
    """X and Y carry orthogonal Hadamard rows of equal power: XY = YX = 0."""
    H = np.array([[1]])
    while H.shape[0] < 64:
        H = np.block([[H, H], [H, -H]])
    x, y = 5 * H[3].astype(complex), 5 * H[10].astype(complex)
    I, Q, U, V = _auto_stokes(x, y)
    assert (I, Q, U, V) == (2 * 25 * 64, 0, 0, 0)


def test_fully_polarised_invariant():
    """x_Y = c x_X with a Gaussian-integer c: I^2 = Q^2 + U^2 + V^2 exactly."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        s = _sig(32, int(rng.integers(1 << 30)))
        c = complex(int(rng.integers(-3, 4)), int(rng.integers(-3, 4)))
        x_y = s * c
        if np.abs(x_y.real).max() > 127 or np.abs(x_y.imag).max() > 127:
            continue
        I, Q, U, V = _auto_stokes(s, x_y)
        assert I.imag == Q.imag == U.imag == V.imag == 0
        assert I.real ** 2 == Q.real ** 2 + U.real ** 2 + V.real ** 2


def test_cross_feed_products_from_voltages():
    """Three feeds: every feed pair's Stokes equals the combination of
    products sum_t x_p conj(x_q) formed directly from the voltages."""
    rng = np.random.default_rng(9)
    nf, T = 3, 40
    x = rng.integers(-30, 31, (2 * nf, T)) + 1j * rng.integers(-30, 31, (2 * nf, T))
    S = st.stokes(_vis(x), 2 * nf)[0]
    for a in range(nf):
        for b in range(a + 1):
            prod = {}
            for pa, na in ((0, "X"), (1, "Y")):
                for pb, nb in ((0, "X"), (1, "Y")):
                    prod[na + nb] = np.sum(x[2 * a + pa] * np.conj(x[2 * b + pb]))
            want = [prod["XX"] + prod["YY"], prod["XX"] - prod["YY"], prod["XY"] + prod["YX"],
                    -1j * (prod["XY"] - prod["YX"])]
            p = a * (a + 1) // 2 + b
            got = S[p, :, 0] + 1j * S[p, :, 1]
            assert np.array_equal(got, np.array(want)), (a, b)


def test_odd_input_count_refused():
    with pytest.raises(ValueError):
        st.stokes(np.zeros((1, 6, 2), np.int32), 3)


# planted mistakes in copies of the oracle, each of which some pin must catch
MUTANTS = [
    ("v_sign_flipped", "out[:, p, 3, 0] = d[:, 1]", "out[:, p, 3, 0] = -d[:, 1]"),
    ("q_is_yy_minus_xx", "out[:, p, 1] = xx - yy", "out[:, p, 1] = yy - xx"),
    ("xy_yx_swapped", "xy = _vis(V, 2 * a, 2 * b + 1)", "xy = _vis(V, 2 * a + 1, 2 * b)"),
    ("no_conjugate_above_diagonal", "return np.stack([v[:, 0], -v[:, 1]], axis=-1)", "return v"),
    ("pols_swapped", "yy = _vis(V, 2 * a + 1, 2 * b + 1)", "yy = _vis(V, 2 * a, 2 * b)"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new, monkeypatch):
    import types
    src = open(st.__file__).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType("stokes_" + name)
    exec(compile(src.replace(old, new), f"<{name}>", "exec"), mod.__dict__)
    monkeypatch.setattr(st, "stokes", mod.stokes)
    pins = [test_textbook_states, test_orthogonal_codes_are_unpolarised, test_fully_polarised_invariant,
            test_cross_feed_products_from_voltages]
    caught = []
    for pin in pins:
        try:
            pin()
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"no pin caught '{name}'"
