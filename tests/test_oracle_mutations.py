"""Mutation check of the oracle's pins (CPU only).

Each mutant below is a plausible mistake in the FP64 oracle: a convention of Section 2
eq. (IQUV) or Section 2.1 read differently, an epsilon of Tables 1-2 misplaced, a comparison
direction flipped, a flag applied to the wrong samples, a term of the pairwise moment update
dropped, the 16-bit sums of Table 4 done in 32 bit.  The oracle is patched with the mutant
and every pin listed for it must then fail, while the same pins pass on the unpatched oracle.
For the conventions that window C separates, the mutant must also reproduce the value that
convention gives (the "must not be produced" values of the pins), so those values are checked
to be what the wrong readings compute.
"""
import importlib
import math

import numpy as np
import pytest

import oracle
from tests import test_oracle_mixed as mixed_pins
from tests import test_oracle_pins as pins

SCREEN = importlib.import_module("oracle.screen")
MIXED = importlib.import_module("oracle.mixed")
EPS = 2.0 ** -23

_orig = {name: getattr(SCREEN, name) for name in ("stokes", "sk_tau", "ds_r", "flag_bits", "masked_average",
                                                   "window_view")}
_orig_update = SCREEN.AdaptiveState.update
_orig_seq16 = MIXED._seq_sum16


def _no_j(vis):                       # V = xy - yx (the j of eq. IQUV dropped)
    I, Q, U, V = _orig["stokes"](vis)
    return I, Q, U, -1j * V


def _u_minus(vis):                    # U = xy - yx
    I, Q, U, V = _orig["stokes"](vis)
    return I, Q, -1j * V, V


def _sk_of_power(I, d, eps):          # SK of |I|^2 instead of |I|
    return _orig["sk_tau"](I * np.abs(I), d, eps)


def _table1_bracket(I, d, eps):       # tau = pre W S2 / (S1^2 + eps) - 1
    W = I.shape[-1]
    pre = (W * d + 1.0) / (W - 1.0)
    return _orig["sk_tau"](I, d, eps) + pre - 1.0


def _sk_prefactor(I, d, eps):         # (W d - 1) / (W - 1) in place of (W d + 1) / (W - 1)
    W = I.shape[-1]
    return _orig["sk_tau"](I, d, eps) * (W * d - 1.0) / (W * d + 1.0)


def _no_eps_in_s1(I, d, eps):         # S1^2 without the epsilon of Table 1 group 7
    return _orig["sk_tau"](I, d, 0.0)


def _eps_under_sqrt(q, u, v, eps):    # p = sqrt(q^2 + u^2 + v^2 + eps)
    W = q.shape[-1]
    p = np.sqrt(q * q + u * u + v * v + eps)
    return np.sqrt((q / p).sum(-1) ** 2 + (u / p).sum(-1) ** 2 + (v / p).sum(-1) ** 2) / W


def _r_over_w_minus_1(q, u, v, eps):
    W = q.shape[-1]
    return _orig["ds_r"](q, u, v, eps) * W / (W - 1.0)


def _ge_for_gt(tau, r_re, r_im, s_low, s_high, gamma, options=0, gamma_im=None):   # SK_HIGH on tau >= s_high
    bits = _orig["flag_bits"](tau, r_re, r_im, s_low, s_high, gamma, options, gamma_im)
    if not options & oracle.OPT_NO_SK:
        bits = bits | np.where(np.asarray(tau, np.float64) == s_high, oracle.SK_HIGH, 0).astype(np.uint8)
    return bits


def _mask_reversed(vis, flags, M, F=1):   # each flag applied to the wrong window
    return _orig["masked_average"](vis, np.asarray(flags)[..., ::-1], M, F)


def _mask_times_zero(vis, flags, M, F=1):  # flagged samples multiplied by 0 instead of left out
    v = oracle.as_complex128(vis)
    keep = np.repeat(np.repeat(np.asarray(flags) == 0, F, axis=-2), M, axis=-1)
    n = keep.sum(axis=-1)
    with np.errstate(invalid="ignore", divide="ignore"):
        total = (v * keep[..., None]).sum(axis=-2)
        avg = np.where(n[..., None] > 0, total / np.maximum(n, 1)[..., None], 0.0)
    return avg, n / v.shape[-2]


def _window_time_major(vis, M, F=1):  # F channels' windows taken as F M consecutive samples of one channel
    v = oracle.as_complex128(vis)
    *lead, C, T, four = v.shape
    v = v.reshape(*lead, C // F, F * T, 4)
    return v.reshape(*lead, C // F, T // M, F * M, 4)


def _update_no_cross(self, stats, keep):  # Chan's update without the delta^2 n n_b / n' term
    m2_before = self.m2.copy()
    n_before = self.n.astype(np.float64)
    kb = keep.astype(np.float64)
    nb = kb.sum(axis=-1)
    with np.errstate(invalid="ignore", divide="ignore"):
        mb = (stats * kb[..., None]).sum(axis=-2) / np.maximum(nb, 1)[..., None]
    delta = mb - self.mean
    cross = np.where(nb > 0, n_before * nb / np.maximum(n_before + nb, 1), 0.0)[..., None]
    _orig_update(self, stats, keep)
    self.m2 = self.m2 - delta * delta * cross
    assert self.m2.shape == m2_before.shape


def _seq_sum32(x):                    # Table 4 group 4 summed in float32, rounded to binary16 once
    acc = np.zeros(x.shape[:-1], np.float32)
    for i in range(x.shape[-1]):
        acc = (acc + x[..., i]).astype(np.float32)
    return acc.astype(np.float16)


# mutant -> (what it patches, the pins that must catch it)
MUTANTS = {
    "V without j": ({"stokes": _no_j}, [
        (pins.test_stokes_are_pauli_traces, ()),
        (pins.test_su2_invariance_of_all_statistics, ()),
        (pins.test_worked_window_C_high_precision, (1.0,))]),
    "U = xy - yx": ({"stokes": _u_minus}, [(pins.test_stokes_are_pauli_traces, ())]),
    "SK of |I|^2": ({"sk_tau": _sk_of_power}, [
        (pins.test_sk_unit_mean_and_variance_on_gamma_inputs, (1, 16, 200_000)),
        (pins.test_worked_window_C_high_precision, (1.0,))]),
    # (at d = 0.5 and W = 4 the prefactor is 1 and the two brackets agree: d = 1 separates them)
    "Table 1 one-line bracket": ({"sk_tau": _table1_bracket}, [
        (pins.test_sk_constant_window, (4, 1.0)),
        (pins.test_worked_window_C_high_precision, (1.0,))]),
    "SK prefactor (Wd-1)/(W-1)": ({"sk_tau": _sk_prefactor}, [
        (pins.test_sk_one_hot_is_maximum, (16, 2.2)),
        (pins.test_worked_window_B_one_hot, (1.0,))]),
    "no eps in S1^2": ({"sk_tau": _no_eps_in_s1}, [(pins.test_sk_constant_window, (16, 2.2))]),
    "eps under the sqrt": ({"ds_r": _eps_under_sqrt}, [
        (pins.test_worked_window_A_constant, (1.0,)),
        (pins.test_ds_identical_directions, ())]),
    "r / (W - 1)": ({"ds_r": _r_over_w_minus_1}, [
        (pins.test_worked_window_B_one_hot, (0.5,)),
        (pins.test_ds_isotropic_null_second_moment, (16,))]),
    ">= for > (SK high)": ({"flag_bits": _ge_for_gt}, [(pins.test_flag_bits_brute_force, (2.0, 0.0, 0.0, 0))]),
    "flags on the wrong windows": ({"masked_average": _mask_reversed}, [
        (pins.test_masked_average_library_cross_check, ()),
        (pins.test_masked_average_worked_example, ())]),
    "flagged samples times zero": ({"masked_average": _mask_times_zero}, [
        (pins.test_nonfinite_input_flags_window, ())]),
    "time x frequency window time-major": ({"window_view": _window_time_major}, [
        (pins.test_time_frequency_window_W20_by_hand, ()),
        (pins.test_time_frequency_window_brute_force, ())]),
    "Chan update without the cross term": ({"AdaptiveState.update": _update_no_cross}, [
        (pins.test_adaptive_state_matches_numpy_moments, ())]),
    "Table 4 sums in 32 bit": ({"mixed._seq_sum16": _seq_sum32}, [
        (mixed_pins.test_binary16_unit_vector_sums_by_hand, ())]),
}


def _apply(monkeypatch, patch):
    for name, fn in patch.items():
        if name == "AdaptiveState.update":
            monkeypatch.setattr(SCREEN.AdaptiveState, "update", fn)
        elif name == "mixed._seq_sum16":
            monkeypatch.setattr(MIXED, "_seq_sum16", fn)
        else:
            monkeypatch.setattr(SCREEN, name, fn)
            monkeypatch.setattr(oracle, name, fn)
            if hasattr(MIXED, name):
                monkeypatch.setattr(MIXED, name, fn)


def _fails(fn, args):
    try:
        fn(*args)
    except Exception:        # an assertion, or any error the mistake provokes
        return True
    return False


@pytest.mark.parametrize("name", list(MUTANTS))
def test_every_mutant_fails_its_pins(name, monkeypatch):
    patch, checks = MUTANTS[name]
    for fn, args in checks:
        assert not _fails(fn, args), f"{fn.__name__}{args} fails on the unpatched oracle"
    with monkeypatch.context() as m:
        _apply(m, patch)
        survived = [f"{fn.__name__}{args}" for fn, args in checks if not _fails(fn, args)]
    assert not survived, f"mutant '{name}' passes {survived}"


def test_wrong_conventions_give_the_values_window_C_excludes(monkeypatch):
    """The must-not-be-produced values of window C are what the wrong readings compute."""
    win = pins.WIN_C
    with monkeypatch.context() as m:
        _apply(m, {"stokes": _no_j})
        _, rre, rim = pins._stats(win, 1.0)
        assert (rre[0], rim[0]) == pytest.approx(pins.C_WRONG["V without j (r_re, r_im)"], rel=1e-12)
    with monkeypatch.context() as m:
        _apply(m, {"sk_tau": _sk_of_power})
        tau, _, _ = pins._stats(win, 1.0)
        assert tau[0] == pytest.approx(pins.C_WRONG["SK of |I|^2 (tau, d = 1)"], rel=1e-12)
    with monkeypatch.context() as m:
        _apply(m, {"sk_tau": _table1_bracket})
        tau, _, _ = pins._stats(win, 1.0)
        assert tau[0] == pytest.approx(pins.C_WRONG["Table 1 one-line bracket (tau, d = 1)"], rel=1e-12)
    assert not math.isnan(pins.C_R_RE)
