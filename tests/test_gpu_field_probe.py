"""Element-wise probe of the field of eqs. (4)/(5) on every plan, at the bench
size N = 2000, R = 1024, every replica and every spin (marked `gpu`).

One step with a0 = 0, gamma = 0, c0 = dt = 1 and y0 = 0 leaves x unchanged and
gives y1 = fl32(f) exactly: p = a0 - a(t_0) = 0, so eq. (16) is y~ = c0 f dt = f,
eq. (17) is x~ = x, no wall is hit (|x| < 1), and eq. (22) adds gamma y dt = 0.
The probe compares each of the 2,048,000 elements of y1 with the oracle's FP64
field of the same x:

  * dSB with +-1 couplings (every plan, the incremental one included) and any
    plan on x on a coarse grid (multiples of 2^-7, |x| <= 12 2^-7): every
    product and partial sum is exact in FP32, so y1 must equal the field
    bit for bit.  This pins each plan's operand encoding (signs, base-8 FP4
    digits and block scales, int8 digits), its layout and its products on
    every element.
  * bSB from the seeded state (24-bit mantissas), against each plan's
    error model:
      - integer-digit plan, integer J: the exactly rounded field of the
        digit representation q = rint(x 2^30) 2^-30 (x itself for
        |x| >= 2^-6):  |y1 - f| <= u |f| + (1 + u) sum_{|x_j| < 2^-6} |J_ij| 2^-31;
      - FP4 plan: the representation of x by eight base-8 digits of its
        32-spin chunk c (to 2^(E_c - 23) <= 2^-22 M_c, M_c = max_c |x|), plus one
        rounding per accumulation of a digit product (8 per 64-spin block,
        blocks in order) of partial sums no larger than S_i:
          |y1 - f| <= 2^-22 sum_j |J_ij| M_c(j) + 8 nkb u S_i,
          S_i = max_b |F_ib| + max_b sum_{j in b} |J_ij| (|x_j| + 2.3 M_c(j)) + rep,
        F_ib the field of the first b blocks;
      - FP32 plan: recursive FP32 summation, |y1 - f| <= gamma_N sum_j |J_ij x_j|;
  * Gaussian couplings (four per-row-scaled int8 digits of J, s_i <= 2 max_j
    |J_ij| the row's power-of-two scale): the representation of J (s_i 2^-31
    per entry), of x (2^-31 below 2^-6), the digit products left out (weights
    a + b >= 4: at most 3.008 2^-30 s_i per spin) and one final rounding.

u = 2^-24 is the unit roundoff of single precision.  Every case also meets the
bar of a one-step bSB trajectory: per replica ||y1 - f|| / ||f|| <= 1e-5.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_08361_amd import hsb  # noqa: E402

N, R = 2000, 1024
U = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    hsb.load_library()


def say(*a):
    print("[case]", *a, flush=True)


_cache = {}


def instance(kind):
    if kind not in _cache:
        J = synth.sk_instance(N, 2000) if kind == "sk" else synth.gaussian_instance(N, 3)
        _cache[kind] = (J, J.astype(np.float64))
    return _cache[kind]


def start_state(kind):
    """'seeded': the library's own seeded state (amp 0.1, replicas 0..R-1 of
    seed 5).  'grid': multiples of 2^-7 in [-12 2^-7, 12 2^-7] (seeded)."""
    if kind not in _cache:
        if kind == "seeded":
            x0, _ = oracle.init_state(5, R, N, amp=0.1)
        else:
            m = np.random.default_rng(7).integers(-12, 13, size=(R, N))
            x0 = (m * 2.0 ** -7).astype(np.float32)
        _cache[kind] = x0
    return _cache[kind]


def oracle_field(jkind, xkind, variant):
    key = ("f", jkind, xkind, variant)
    if key not in _cache:
        _, J64 = instance(jkind)
        X = start_state(xkind)
        _cache[key] = np.stack([oracle.field(J64, X[r], variant) for r in range(R)])
    return _cache[key]


def probe(jkind, xkind, variant, plan):
    """y1 of the probe step (see the module docstring) and the plan that ran."""
    J, _ = instance(jkind)
    x0 = start_state(xkind)
    with hsb.Context(J, precision=plan) as ctx:
        out = ctx.run_ex(variant, 1, R, 0.0, 1.0, 1.0, 0.0, 0, x0=torch.from_numpy(x0),
                         y0=torch.zeros((R, N), dtype=torch.float32), want_state=True)
        torch.cuda.synchronize()
        x1 = out["x"].cpu().numpy()
        y1 = out["y"].cpu().numpy().astype(np.float64)
        ran = ctx.last_plan()
    assert np.array_equal(x1, x0), "x must not move when a0 = 0"
    return y1, ran


def l2_bar(y1, f):
    rel = np.linalg.norm(y1 - f, axis=1) / np.linalg.norm(f, axis=1)
    assert rel.max() <= 1e-5, rel.max()


DSB_PLANS = [("fp32", "fp32"), ("mixed", "fp4"), ("digits", "digits"),
             ("incremental", "incremental")]


@pytest.mark.parametrize("plan,expect", DSB_PLANS)
def test_dsb_field_every_element_exact(plan, expect):
    say("field probe dsb sk", plan)
    y1, ran = probe("sk", "seeded", hsb.HSB_DSB, plan)
    assert ran == expect
    f = oracle_field("sk", "seeded", oracle.DSB)
    bad = np.argwhere(y1 != f)
    assert bad.size == 0, (len(bad), bad[:5])


@pytest.mark.parametrize("plan,expect", [("fp32", "fp32"), ("mixed", "fp4"), ("digits", "digits")])
def test_bsb_field_on_grid_every_element_exact(plan, expect):
    say("field probe bsb sk grid", plan)
    y1, ran = probe("sk", "grid", hsb.HSB_BSB, plan)
    assert ran == expect
    f = oracle_field("sk", "grid", oracle.BSB)
    bad = np.argwhere(y1 != f)
    assert bad.size == 0, (len(bad), bad[:5])


def chunk_max(X):
    """M_c(j): max |x| over the 32-spin chunk of spin j, per replica."""
    Np = -(-N // 32) * 32
    A = np.zeros((X.shape[0], Np))
    A[:, :N] = np.abs(X)
    M = A.reshape(X.shape[0], -1, 32).max(axis=2)
    return np.repeat(M, 32, axis=1)[:, :N]


def fp4_bound(J64, X, f):
    """Per-element bound of the FP4 plan's bSB field (module docstring)."""
    Xd = X.astype(np.float64)
    Mc = chunk_max(Xd)
    A = np.abs(J64)
    rep = Mc @ A.T * 2.0 ** -22                     # [R][N]: sum_j |J_ij| M_c(j)
    nkb = -(-N // 256) * 4                          # 64-spin blocks of the padded size
    Np = nkb * 64
    # largest prefix field over whole blocks (blocks in natural order)
    Fmax = np.zeros_like(f)
    acc = np.zeros_like(f)
    blk = np.zeros_like(f)
    W = np.abs(Xd) + 2.3 * Mc
    for b in range(0, N, 64):
        e = min(b + 64, N)
        acc += Xd[:, b:e] @ J64[:, b:e].T
        Fmax = np.maximum(Fmax, np.abs(acc))
        blk = np.maximum(blk, W[:, b:e] @ A[:, b:e].T)
    assert Np >= N
    S = Fmax + blk + rep
    return rep + 8 * nkb * U * S


@pytest.mark.parametrize("plan,expect", [("fp32", "fp32"), ("mixed", "fp4"), ("digits", "digits")])
def test_bsb_field_seeded_within_error_model(plan, expect):
    say("field probe bsb sk seeded", plan)
    y1, ran = probe("sk", "seeded", hsb.HSB_BSB, plan)
    assert ran == expect
    J, J64 = instance("sk")
    X = start_state("seeded")
    f = oracle_field("sk", "seeded", oracle.BSB)
    err = np.abs(y1 - f)
    A = np.abs(J64)
    if expect == "digits":
        small = (np.abs(X) < 2.0 ** -6).astype(np.float64)
        bound = U * np.abs(f) + (1 + U) * (small @ A.T) * 2.0 ** -31 + 1e-300
    elif expect == "fp4":
        bound = fp4_bound(J64, X, f)
    else:
        gN = N * U / (1 - N * U)
        bound = gN * (np.abs(X.astype(np.float64)) @ A.T)
    ratio = err / bound
    say("  max |err|", err.max(), "max err/bound", ratio.max(), "median", np.median(ratio))
    assert np.all(err <= bound), np.unravel_index(np.argmax(ratio), ratio.shape)
    l2_bar(y1, f)


def gaussian_digit_bound(J64, X, f, variant):
    A = np.abs(J64)
    s = 2.0 * A.max(axis=1)                         # >= the row's power-of-two scale
    Xd = X.astype(np.float64)
    B = np.abs(Xd) if variant == oracle.BSB else np.ones_like(Xd)
    jrep = (B.sum(axis=1)[:, None] * s[None, :]) * 2.0 ** -31
    if variant == oracle.BSB:
        small = (np.abs(Xd) < 2.0 ** -6).astype(np.float64)
        xrep = (small @ A.T) * 2.0 ** -31
        drop = (N - 1) * 3.008 * 2.0 ** -30 * s[None, :]
    else:
        xrep = drop = 0.0
    return U * np.abs(f) + (1 + U) * (jrep + xrep + drop) * (1 + 1e-9)


@pytest.mark.parametrize("variant", [hsb.HSB_BSB, hsb.HSB_DSB])
@pytest.mark.parametrize("plan,expect", [("fp32", "fp32"), ("digits", "digits")])
def test_gaussian_field_within_error_model(variant, plan, expect):
    say("field probe gaussian", variant, plan)
    y1, ran = probe("gauss", "seeded", variant, plan)
    assert ran == expect
    J, J64 = instance("gauss")
    X = start_state("seeded")
    ov = oracle.BSB if variant == hsb.HSB_BSB else oracle.DSB
    f = oracle_field("gauss", "seeded", ov)
    err = np.abs(y1 - f)
    if expect == "digits":
        bound = gaussian_digit_bound(J64, X, f, ov)
    else:
        gN = N * U / (1 - N * U)
        B = np.abs(X.astype(np.float64)) if ov == oracle.BSB else np.ones(X.shape)
        bound = gN * (B @ np.abs(J64).T)
    ratio = err / bound
    say("  max |err|", err.max(), "max err/bound", ratio.max())
    assert np.all(err <= bound), np.unravel_index(np.argmax(ratio), ratio.shape)
    l2_bar(y1, f)
