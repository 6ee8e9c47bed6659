"""Error bounds that the BF16 Panther++ form relies on (Sec. 3.3 distances
over bfloat16 copies of theta), checked on the CPU by emulating the FP32
evaluation order of the pool pass.

* d2~ = fl(fl(|b_v|^2 - 2 <b_q, b_v>) + |b_q|^2) errs from the exact
  |b_q - b_v|^2 by at most 2^-15 (|b_q|^2 + |b_v|^2), in any summation order
  of the 64-term products (checked for sequential, pairwise and reversed
  orders); for integral rows with |b_q|^2 + |b_v|^2 < 2^23 it is exact.
* bfloat16 rounding moves a row by at most 2^-8 of its norm.
* The norm band: a row whose FP32 norm lies outside the query's band for
  threshold t has d2~ > t (so the band search may skip it).

These are the bounds stated where the certificate and the band search are
implemented.  The cases show the bounds hold for count-like rows from 1 to
10^5 per coordinate, that FP32 rounding does occur for large rows (so
treating them as exact would be wrong: about 12 units of 2^-24 of
|b_q|^2 + |b_v|^2 against the 512 allowed), and that no row the band
search skips could have entered a pool; a band with a wrong radius (say
sqrt(t)/2) skips rows inside the threshold and fails.  The rounding
margins of the band are not exercised by random rows.
"""
import numpy as np


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), as float32."""
    a = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((a + 0x7FFF + ((a >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def f32(x):
    return np.float32(x)


def dot32(a, b, order):
    """FP32 sum of the exact float32 products of a and b in a given order."""
    p = (a.astype(np.float32) * b.astype(np.float32)).astype(np.float32)
    if order == "seq":
        s = np.float32(0)
        for x in p:
            s = np.float32(s + x)
        return s
    if order == "rev":
        s = np.float32(0)
        for x in p[::-1]:
            s = np.float32(s + x)
        return s
    # pairwise (a tree, as a matrix core may reduce)
    v = list(p)
    while len(v) > 1:
        v = [np.float32(v[i] + v[i + 1]) if i + 1 < len(v) else v[i]
             for i in range(0, len(v), 2)]
    return v[0]


def d2_tilde(bq, bv, order):
    acc = dot32(bq, bv, order)
    nv = dot32(bv, bv, order)
    qn = dot32(bq, bq, order)
    u = f32(np.float64(nv) - 2.0 * np.float64(acc))  # one rounding (fma)
    return f32(np.float64(u) + np.float64(qn)), qn, nv


def exact_d2(bq, bv):
    d = bq.astype(np.float64) - bv.astype(np.float64)
    return float(np.dot(d, d))


def rows(rng, count, scale):
    """Count-like rows: descending lognormal magnitudes, D = 50, padded to 64."""
    x = np.sort(rng.lognormal(0.0, 1.5, size=(count, 50)) * scale, axis=1)[:, ::-1]
    x = np.floor(x).astype(np.float32)
    return np.concatenate([x, np.zeros((count, 14), np.float32)], axis=1)


def test_d2_error_bound_any_order():
    rng = np.random.default_rng(1)
    worst = 0.0
    for scale in (1.0, 30.0, 1e3, 1e5):
        xs = rows(rng, 40, scale)
        bs = bf16(xs)
        for i in range(0, 40, 2):
            bq, bv = bs[i], bs[i + 1]
            ex = exact_d2(bq, bv)
            bound = 2.0 ** -15 * (float(np.dot(bq.astype(np.float64), bq)) +
                                  float(np.dot(bv.astype(np.float64), bv)))
            for order in ("seq", "rev", "pair"):
                got, _, _ = d2_tilde(bq, bv, order)
                err = abs(float(got) - ex)
                assert err <= bound, (scale, i, order, err, bound)
                if bound > 0:
                    worst = max(worst, err / (bound * 2.0 ** -9))  # in 2^-24 units
    # rounding does occur (an exact-evaluation assumption for large rows
    # would be wrong), and stays far inside the bound (512 units)
    assert 1.0 <= worst < 64.0


def test_d2_exact_for_small_integral_rows():
    rng = np.random.default_rng(2)
    for _ in range(200):
        bq = np.concatenate([rng.integers(0, 256, 50), np.zeros(14)]).astype(np.float32)
        bv = np.concatenate([rng.integers(0, 256, 50), np.zeros(14)]).astype(np.float32)
        assert (bf16(bq) == bq).all() and (bf16(bv) == bv).all()  # counts < 256 stay
        if np.dot(bq.astype(np.float64), bq) + np.dot(bv.astype(np.float64), bv) >= 2 ** 23:
            continue
        for order in ("seq", "pair"):
            got, _, _ = d2_tilde(bq, bv, order)
            assert float(got) == exact_d2(bq, bv)


def test_bf16_rounding_relative_bound():
    rng = np.random.default_rng(3)
    x = (rng.lognormal(0.0, 3.0, size=(500, 64)) * rng.choice([1, 100, 1e4], (500, 1))).astype(
        np.float32)
    b = bf16(x)
    err = np.abs(b.astype(np.float64) - x.astype(np.float64))
    assert (err <= 2.0 ** -8 * np.abs(x.astype(np.float64))).all()
    rn = np.linalg.norm(b.astype(np.float64) - x.astype(np.float64), axis=1)
    assert (rn <= 2.0 ** -8 * np.linalg.norm(x.astype(np.float64), axis=1)).all()


def norm_band(qn, t):
    """The pool pass's band for a query of FP32 norm^2 qn and threshold t."""
    qn = np.float32(qn)
    t = np.float32(t)
    rq = np.float32(np.sqrt(qn))
    rho = np.float32(np.sqrt(np.float32((t + qn * np.float32(2.44140625e-4)) *
                                        np.float32(1 + 2.44140625e-4))))
    hi = np.float32(rq * np.float32(1 + 1.52587890625e-5) + rho)
    lo = np.float32(rq * np.float32(1 - 1.52587890625e-5) - rho)
    hi2 = np.float32(hi * hi * np.float32(1 + 2.44140625e-4))
    lo2 = np.float32(lo * lo * np.float32(1 - 2.44140625e-4)) if lo > 0 else np.float32(0)
    return lo2, hi2


def test_norm_band_skips_only_rows_beyond_threshold():
    rng = np.random.default_rng(4)
    checked = 0
    for scale in (1.0, 50.0, 3e3):
        bs = bf16(rows(rng, 300, scale))
        for i in range(0, 300, 3):
            bq = bs[i]
            # thresholds between the nearest and the median candidate
            cand = [d2_tilde(bq, bs[j], "seq")[0] for j in range(300) if j != i]
            for t in (np.float32(np.quantile(cand, 0.01)), np.float32(np.median(cand))):
                qn = dot32(bq, bq, "seq")
                lo2, hi2 = norm_band(qn, t)
                for j in range(300):
                    if j == i:
                        continue
                    d2, _, nv = d2_tilde(bq, bs[j], "seq")
                    if nv > hi2 or nv < lo2:  # skipped by the band search
                        checked += 1
                        assert d2 > t, (scale, i, j, float(d2), float(t))
    assert checked > 1000
