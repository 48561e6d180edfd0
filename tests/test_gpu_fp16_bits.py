"""The scaled-float16 form stores every value of L and U as the binary16
rounding (round to nearest, ties to even) of (s_l[i] a_ij) s_r[j]; the GPU's
conversion and the oracle's or_round_f16 must agree bit for bit.

The stored values are read back through the apply itself: on a matrix with
unit diagonal (s_l = s_r = 1 exactly), one forward GS2 half with one inner
sweep and w = 1 applied to the unit vector e_j gives, for every row i > j,
z_i = 0 - Lh_ij s_l[j] exactly (a binary16 value widened to binary32, times
+-1, negated; then widened to float64): the stored value itself, bit for
bit (a stored zero is compared by value: the sign of a zero row sum is not
the stored value's).  A backward half
reads Uh the same way.  The values include binary16 subnormals, exact ties
between neighbouring binary16 numbers, and magnitudes up to 65504."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2104_01196_amd as g  # noqa: E402
from gen import CSR  # noqa: E402

pytestmark = pytest.mark.gpu


def special_values(rng, k):
    h = np.arange(1, 0x7BFF, dtype=np.uint16).view(np.float16).astype(np.float64)
    ties = (h[:-1] + h[1:]) / 2                      # exact midpoints: ties to even
    sub = rng.uniform(2.0 ** -26, 2.0 ** -14, k)      # binary16 subnormal range
    big = rng.uniform(1000.0, 65504.0, k)
    mid = rng.standard_normal(k) * 10.0 ** rng.uniform(-6, 3, k)
    vals = np.concatenate([rng.choice(ties, k), sub, big, mid])
    return vals * rng.choice([-1.0, 1.0], vals.size)


def banded_unit_diag(n, offsets, rng, neg_rows):
    """Unit-diagonal matrix (diagonal -1 on neg_rows) with entries on the
    given diagonals; values drawn from special_values."""
    rows, cols = [], []
    for i in range(n):
        for o in sorted(set(offsets) | {0}):
            j = i + o
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
    rows, cols = np.array(rows), np.array(cols)
    vals = special_values(rng, (rows.size + 3) // 4)[: rows.size]
    rng.shuffle(vals)
    vals[rows == cols] = 1.0
    vals[(rows == cols) & np.isin(rows, neg_rows)] = -1.0
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, rows + 1, 1)
    return CSR(n, np.cumsum(rp).astype(np.int32), cols.astype(np.int32), vals)


@pytest.mark.parametrize("fmt", [g.FORMAT_SELL, g.FORMAT_DIA])
def test_fp16_stored_values_equal_oracle_rounding(fmt):
    rng = np.random.default_rng(77)
    n = 320
    A = banded_unit_diag(n, [-1, -2, -9, -40, 1, 3, 17, 50], rng, neg_rows=np.arange(5, n, 37))
    dA = g.DeviceCSR.from_host(A)
    M = A.to_scipy().tocsc()
    d = A.to_scipy().diagonal()
    z = torch.empty(n, dtype=torch.float64, device="cuda")
    v = torch.zeros(n, dtype=torch.float64, device="cuda")
    checked = 0
    for variant in (g.FORWARD, g.BACKWARD):
        h = g.gs2_setup(dA, 1, 1, 1.0, variant, precision=g.FP16_SCALED, format=fmt)
        assert g.gs2_handle_schedule(h)["format"] == fmt
        for j in range(n):
            v.zero_()
            v[j] = 1.0
            g.gs2_apply(h, v, z)
            zh = z.cpu().numpy()
            col = M.getcol(j)
            for i, a in zip(col.indices, col.data):
                if (variant == g.FORWARD and i > j) or (variant == g.BACKWARD and i < j):
                    # scaled value (s_l[i] a_ij) s_r[j] with s_r = 1, s_l = sign(d); the probe
                    # enters as g_j = v_j s_l[j] = sign(d_j), an exact sign flip
                    expect = -oracle.round_f16(np.sign(d[i]) * a) * np.sign(d[j])
                    got = zh[i]
                    if expect == 0.0:
                        # a stored zero (an underflow) adds nothing to the row sum, and the sign of
                        # a zero sum depends on the order in which the kernel adds signed zeros
                        assert got == 0.0, (variant, i, j, a, got, expect)
                    else:
                        assert np.float64(got).tobytes() == np.float64(expect).tobytes(), (
                            variant, i, j, a, got, expect)
                    checked += 1
    assert checked == A.nnz - n
