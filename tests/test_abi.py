"""The C-ABI library on the CPU: it loads, exports every symbol the header
declares, and its host-only entry points (planner, certification constants,
argument checks that precede any launch) behave as documented."""
import ctypes
import os
import re
from fractions import Fraction

import numpy as np
import pytest

import paper_2002_09094_amd as ivf
from paper_2002_09094_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ivf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ivf_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    # and the binding wraps exactly the declared set
    assert sorted(_lib.SIGNATURES) == names


def test_status_strings_and_defaults():
    lib = _lib.get()
    assert lib.ivf_status_str(0) == b"IVF_OK"
    assert lib.ivf_status_str(-2) == b"IVF_ERR_UNSORTED"
    o = _lib.ivf_options()
    lib.ivf_default_options(ctypes.byref(o))
    assert o.valtype == 0 and o.certify == 1 and o.cluster_range == 0


def test_planner():
    p = ivf.plan_shape(100)
    assert p["ranges"] == 1 and p["k_r"] == 100
    p = ivf.plan_shape(10_000)
    assert p["ranges"] * p["k_r"] >= 10_000 and p["k_r"] <= 1024 and p["waves"] == 8
    p = ivf.plan_shape(10_000, valtype="bf16")
    assert p["ranges"] == 8 and p["k_r"] == 1250
    assert p["lds_bytes"] <= 160 * 1024
    p = ivf.plan_shape(50_000)
    assert p["ranges"] >= 40 and p["rescore_ranges"] == p["ranges"] and p["rescore_k_r"] == p["k_r"]
    p = ivf.plan_shape(1000, cluster_range=64)
    assert p["k_r"] <= 64 and p["ranges"] == 16
    with pytest.raises(ivf.IvfError):
        ivf.plan_shape(0)
    with pytest.raises(ivf.IvfError):
        ivf.plan_shape(100, waves_per_wg=17)


def test_build_rejects_bad_arguments_before_any_launch():
    lib = _lib.get()
    h = ctypes.c_void_p()
    # null object set
    assert lib.ivf_build(None, 3, None, ctypes.byref(h)) == -1
    x = _lib.ivf_csr(10, 5, 20, 1, 1, 1)   # dummy non-null pointers, never read
    assert lib.ivf_build(ctypes.byref(x), 11, None, ctypes.byref(h)) == -1   # k > n
    assert lib.ivf_build(ctypes.byref(x), 0, None, ctypes.byref(h)) == -1    # k < 1
    big = _lib.ivf_csr(10, 5, 1 << 31, 1, 1, 1)
    assert lib.ivf_build(ctypes.byref(big), 3, None, ctypes.byref(h)) == -5  # capacity
    o = _lib.ivf_options()
    lib.ivf_default_options(ctypes.byref(o))
    o.valtype = 7
    assert lib.ivf_build(ctypes.byref(x), 3, ctypes.byref(o), ctypes.byref(h)) == -1
    assert b"valtype" in lib.ivf_last_error(None)
    assert h.value is None


def _exact_gamma(n, u):
    return Fraction(n) * u / (1 - Fraction(n) * u)


@pytest.mark.parametrize("vt,us", [("f32", Fraction(1, 2 ** 24)),
                                   ("bf16", Fraction(1, 2 ** 8) + Fraction(1, 2 ** 24) +
                                    Fraction(1, 2 ** 32)),
                                   ("f16", Fraction(1, 2 ** 11) + Fraction(1, 2 ** 24) +
                                    Fraction(1, 2 ** 35))])
@pytest.mark.parametrize("nt", [1, 60, 2000])
@pytest.mark.parametrize("vmax", [0.5, 1.0, 50.0])
def test_cert_constants_follow_recursive_summation_bound(vt, us, nt, vmax):
    c, a, g = ivf.cert_bound(vt, nt, vmax)
    u32 = Fraction(1, 2 ** 24)
    want = (1 + us) * (1 + _exact_gamma(nt, u32)) - 1
    assert c >= float(want) * 1.01 and c <= float(want) * 1.0101 + 1e-14
    assert g >= float(_exact_gamma(nt, Fraction(1, 2 ** 53)))
    # absolute term: per product, the mean value's rounding below the normal
    # range (times the object value) and two FP32 roundings of tiny results
    eta = Fraction(1, 2 ** 126)
    eta_m = eta + (Fraction(1, 2 ** 25) if vt == "f16" else 0)
    a_want = nt * (Fraction(vmax) * eta_m + 2 * eta) * (1 + _exact_gamma(nt, u32))
    assert a >= float(a_want) * 1.01 * (1 - 1e-12) and a <= float(a_want) * 1.0101


def _round_bf16(x32):
    b = x32.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32)


def _round_f32(q):
    """The FP32 value nearest the rational q >= 0 (ties to even), subnormals
    included: a fused multiply-add's single rounding."""
    if q == 0:
        return np.float32(0)
    e = q.numerator.bit_length() - q.denominator.bit_length()
    if Fraction(2) ** e > q:
        e -= 1
    quantum = Fraction(2) ** (max(e, -126) - 23)      # spacing of FP32 values near q
    m = q / quantum
    r = m.numerator // m.denominator
    rem = m - r
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and r % 2 == 1):
        r += 1
    return np.float32(float(r * quantum))


def test_round_f32_matches_numpy_on_doubles():
    rng = np.random.default_rng(5)
    for x in np.concatenate([rng.uniform(0, 1, 2000) ** 9, [2.0 ** -149, 3 * 2.0 ** -150, 1.0]]):
        assert _round_f32(Fraction(float(x))) == np.float32(x)


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("vt", ["f32", "bf16", "f16"])
def test_cert_bound_holds_for_emulated_fp32_scores(vt, fused):
    """Emulate the tile arithmetic on the CPU (mean value rounded to the stored
    precision, then either an FP32 product added with a second rounding or a
    fused multiply-add rounded once, summed in order) and check the stated
    bound against the exact score, including adversarial magnitudes.  The
    16-bit walks accumulate fused, the FP32 walk unfused."""
    rng = np.random.default_rng(3)
    for trial in range(300):
        nt = int(rng.integers(1, 400))
        v = rng.uniform(0, 1, nt) ** rng.uniform(1, 8)
        v = (v / np.linalg.norm(v)).astype(np.float32)
        v[v == 0] = np.float32(1e-30)
        u = (rng.uniform(0, 1, nt) ** rng.uniform(1, 12)) * 10.0 ** -rng.uniform(0, 6)
        u = u.astype(np.float64)
        u32 = u.astype(np.float32)
        if vt == "bf16":
            us = _round_bf16(u32)
        elif vt == "f16":
            us = u32.astype(np.float16).astype(np.float32)
        else:
            us = u32
        acc = np.float32(0)
        for t in range(nt):
            if fused:
                acc = _round_f32(Fraction(float(acc)) + Fraction(float(v[t])) * Fraction(float(us[t])))
            else:
                acc = np.float32(acc + np.float32(v[t] * us[t]))
        exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(v, u))
        c, a, _ = ivf.cert_bound(vt, nt, float(v.max()))
        err = abs(Fraction(float(acc)) - exact)
        assert err <= Fraction(c) * exact + Fraction(a), (vt, trial, float(err), float(exact))


def test_cert_bound_holds_for_split_fp32_sums():
    """The FP32 register walk sums an object's dense-slab products and its
    sparse-slice products separately (each in ascending term order) and adds
    the two once.  Emulate that order on the CPU, with an arbitrary split of
    the terms, and check the same bound against the exact score, including
    the adversarial magnitudes of the sequential test."""
    rng = np.random.default_rng(29)
    for trial in range(300):
        nt = int(rng.integers(1, 400))
        v = rng.uniform(0, 1, nt) ** rng.uniform(1, 8)
        v = (v / np.linalg.norm(v)).astype(np.float32)
        v[v == 0] = np.float32(1e-30)
        u = (rng.uniform(0, 1, nt) ** rng.uniform(1, 12)) * 10.0 ** -rng.uniform(0, 6)
        us = u.astype(np.float32)
        dense = rng.uniform(0, 1, nt) < rng.uniform(0, 1)
        acc_d = np.float32(0)
        acc_s = np.float32(0)
        for t in range(nt):
            p = np.float32(v[t] * us[t])
            if dense[t]:
                acc_d = np.float32(acc_d + p)
            else:
                acc_s = np.float32(acc_s + p)
        acc = np.float32(acc_d + acc_s)
        exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(v, u))
        c, a, _ = ivf.cert_bound("f32", nt, float(v.max()))
        err = abs(Fraction(float(acc)) - exact)
        assert err <= Fraction(c) * exact + Fraction(a), (trial, float(err), float(exact))


def _stored(vt, u):
    u32 = u.astype(np.float32)
    if vt == "bf16":
        return _round_bf16(u32)
    if vt == "f16":
        return u32.astype(np.float16).astype(np.float32)
    return u32


def _emulate(vt, v, u, fused):
    us = _stored(vt, u)
    acc = np.float32(0)
    for t in range(len(v)):
        if fused:
            acc = _round_f32(Fraction(float(acc)) + Fraction(float(v[t])) * Fraction(float(us[t])))
        else:
            acc = np.float32(acc + np.float32(v[t] * us[t]))
    return acc


@pytest.mark.parametrize("vt,fused", [("f32", False), ("bf16", True), ("f16", True)])
def test_cert_bound_holds_below_the_normal_range(vt, fused):
    """Adversarial magnitudes below FP32's (or FP16's) normal range: mean
    values that round to subnormals, products that underflow, and object
    values far above 1 beside FP16 subnormal mean values.  The stated bound
    must hold for every emulated sum, and the purely relative part alone must
    fail on some of them (so the absolute term is what carries them)."""
    rng = np.random.default_rng(17)
    relative_alone_fails = 0
    for trial in range(240):
        nt = int(rng.integers(1, 120))
        case = trial % 3
        if case == 0:        # mean values in FP32's subnormal range
            v = (rng.uniform(0.01, 1, nt) / np.sqrt(nt)).astype(np.float32)
            u = 10.0 ** rng.uniform(-45, -37, nt)
        elif case == 1:      # tiny object values: products underflow
            v = (10.0 ** rng.uniform(-30, -20, nt)).astype(np.float32)
            u = 10.0 ** rng.uniform(-25, -5, nt)
        else:                # large object values, mean values below FP16's normal range
            v = rng.uniform(0.5, 50.0, nt).astype(np.float32)
            u = 10.0 ** rng.uniform(-9, -4.3, nt)
        u = u.astype(np.float64)
        acc = _emulate(vt, v, u, fused)
        exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(v, u))
        c, a, _ = ivf.cert_bound(vt, nt, float(v.max()))
        err = abs(Fraction(float(acc)) - exact)
        assert err <= Fraction(c) * exact + Fraction(a), (vt, trial, float(err), float(exact))
        relative_alone_fails += err > Fraction(c) * exact
    assert relative_alone_fails > 0


def test_batch_build_failure_keeps_its_message():
    """A HIP failure while a batch is built (here: no GPU, so the first HIP
    call fails) returns IVF_ERR_HIP, no batch, and a message naming the call."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("needs a machine without a usable GPU")
    lib = _lib.get()
    b = ctypes.c_void_p()
    xs = (_lib.ivf_csr * 1)(_lib.ivf_csr(10, 5, 20, 1, 1, 1))
    ks = (ctypes.c_int32 * 1)(3)
    assert lib.ivf_batch_build(1, xs, ks, None, ctypes.byref(b)) == -7
    assert b.value is None
    assert lib.ivf_batch_last_error(None).startswith(b"hip")


def test_batch_build_rejects_bad_arguments_before_any_launch():
    lib = _lib.get()
    b = ctypes.c_void_p()
    xs = (_lib.ivf_csr * 2)(_lib.ivf_csr(10, 5, 20, 1, 1, 1), _lib.ivf_csr(8, 5, 20, 1, 1, 1))
    ks = (ctypes.c_int32 * 2)(3, 9)                      # k > n in the second instance
    assert lib.ivf_batch_build(2, xs, ks, None, ctypes.byref(b)) == -1
    assert b"k outside" in lib.ivf_batch_last_error(None)
    assert lib.ivf_batch_build(0, xs, ks, None, ctypes.byref(b)) == -1
    assert lib.ivf_batch_build(2, None, ks, None, ctypes.byref(b)) == -1
    big = (_lib.ivf_csr * 1)(_lib.ivf_csr(10, 5, 1 << 31, 1, 1, 1))
    k1 = (ctypes.c_int32 * 1)(3)
    assert lib.ivf_batch_build(1, big, k1, None, ctypes.byref(b)) == -5
    assert b.value is None
    assert lib.ivf_batch_set_slack(None, 0.5, 0) == -1
    lib.ivf_batch_destroy(None)                           # no-op


@pytest.mark.parametrize("below", [0, 7, 19])
def test_fixed_point_bound_holds_for_emulated_ivfd_scores(below):
    """Emulate IVFD's fixed-point scores on the CPU (mean value rounded to
    FP32, FP32 product, product times 2^F rounded to the nearest integer,
    exact integer sum, FP32 conversion, times 2^-F) and check the stated bound
    against the exact score, with adversarial magnitudes, including products
    far below 2^-F.  F is the library's choice from the two norms
    (2^F |x| |mu| <= 2^31), or `below` bits less."""
    rng = np.random.default_rng(5 + below)
    for trial in range(300):
        nt = int(rng.integers(1, 400))
        v = rng.uniform(0, 1, nt) ** rng.uniform(1, 8)
        v = (v / np.linalg.norm(v)).astype(np.float32)
        v[v == 0] = np.float32(1e-30)
        u = (rng.uniform(0, 1, nt) ** rng.uniform(1, 12)) * 10.0 ** -rng.uniform(0, 6)
        u32 = u.astype(np.float32)
        norms = float(np.linalg.norm(v.astype(np.float64))) * float(np.linalg.norm(u))
        F = 31 - int(np.ceil(np.log2(norms * (1 + 2.0 ** -20)))) - below
        S = np.float32(2.0 ** F)
        q = 0
        for t in range(nt):
            p = np.float32(v[t] * u32[t])
            q += int(np.rint(np.float32(p * S)))          # round half to even, as v_rndne
        assert q < 2 ** 32
        got = Fraction(float(np.float32(q))) / Fraction(2) ** F
        exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(v, u))
        c, a, g = ivf.cert_bound_fixed(nt, 2.0 ** F, float(v.max()))
        err = abs(got - exact)
        assert err <= Fraction(c) * exact + Fraction(a), (F, trial, float(err), float(exact))


def test_fixed_point_constants_and_arguments():
    c, a, g = ivf.cert_bound_fixed(100, 2.0 ** 30, 3.0)
    u = Fraction(1, 2 ** 24)
    assert c >= float(((1 + u) ** 3 - 1) * Fraction(101, 100))
    assert a >= 100 * (0.5 / 2 ** 30 + 4.0 * 2.0 ** -126) * 1.01
    assert g >= float(_exact_gamma(100, Fraction(1, 2 ** 53)))
    lib = _lib.get()
    out = (ctypes.c_double * 3)()
    assert lib.ivf_cert_bound_fixed(-1, 1.0, 1.0, out) == -1
    assert lib.ivf_cert_bound_fixed(5, 0.0, 1.0, out) == -1
    assert lib.ivf_cert_bound_fixed(5, float("inf"), 1.0, out) == -1
    assert lib.ivf_cert_bound_fixed(5, 1.0, -1.0, out) == -1
    assert lib.ivf_cert_bound(0, 5, float("nan"), out) == -1
