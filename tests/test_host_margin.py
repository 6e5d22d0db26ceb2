"""The FP32 distance tests of the list build are widened by 16 2^-24 (Q + rs)
(Q bounds every coordinate, rs is the list radius), stated to be twice a
bound on the rounding of the FP32 distance.  This checks that bound on the
host: the kernel's FP32 steps (conversion of FP64 coordinates, difference,
minimum image against the FP32 box side, squared sum, with or without fused
multiply-adds) emulated in numpy, against the exact FP64 distance, on
coordinates up to Q, including pairs across periodic faces and far outside a
free boundary.  (The kernel subtracts the +-L of a stencil cell reached
across a periodic face rather than choosing the image by value; for every
pair within the list radius that is this minimum image, in the same two
roundings.)"""
import numpy as np

U = 2.0 ** -24


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def _fma32(a, b, c):
    # a*b is exact in FP64 for FP32 operands; one rounding to FP32 after the add
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def _min_image32(d, L):
    L = np.float32(L)
    h = np.float32(0.5) * L
    return np.where(d > h, d - L, np.where(d < -h, d + L, d)).astype(np.float32)


def _dist_fp32(qi, qj, box, periodic, fused):
    d = []
    for k in range(3):
        dk = (_f32(qi[:, k]) - _f32(qj[:, k])).astype(np.float32)
        if periodic[k]:
            dk = _min_image32(dk, box[k])
        d.append(dk)
    if fused:
        s = _fma32(d[1], d[1], (d[2] * d[2]).astype(np.float32))
        s = _fma32(d[0], d[0], s)
    else:
        s = ((d[0] * d[0]).astype(np.float32) + (d[1] * d[1]).astype(np.float32)).astype(np.float32)
        s = (s + (d[2] * d[2]).astype(np.float32)).astype(np.float32)
    return np.sqrt(s.astype(np.float64))


def _dist_exact(qi, qj, box, periodic):
    d = qi - qj
    for k in range(3):
        if periodic[k]:
            d[:, k] -= box[k] * np.round(d[:, k] / box[k])
    return np.sqrt((d * d).sum(axis=1))


def _pairs(rng, n, box, periodic, rs, far=0.0):
    box = np.asarray(box, dtype=np.float64)
    qi = rng.random((n, 3)) * box
    # neighbours within ~1.2 rs, some across periodic faces
    qj = qi + (rng.random((n, 3)) - 0.5) * 2.4 * rs / np.sqrt(3.0)
    for k in range(3):
        if periodic[k]:
            qj[:, k] %= box[k]
    if far:
        m = n // 4
        shift = rng.choice([-far, far + box[0]], size=m)
        qi[:m, 0] += shift
        qj[:m, 0] += shift
    return qi, qj


def test_fp32_distance_error_within_half_the_margin():
    rng = np.random.default_rng(11)
    rs = 1.3
    cases = [((70.44, 70.44, 70.44), (1, 1, 1), 0.0),
             ((400.0, 20.0, 20.0), (0, 1, 1), 0.0),
             ((24.0, 8.0, 8.0), (0, 1, 1), 900.0),
             ((6.93, 6.93, 6.93), (1, 1, 1), 0.0)]
    for box, periodic, far in cases:
        qi, qj = _pairs(rng, 200000, box, periodic, rs, far)
        Q = max(max(box), np.abs(qi).max(), np.abs(qj).max())
        bound = 8.0 * U * (Q + rs)
        r = _dist_exact(qi.copy(), qj.copy(), box, periodic)
        near = r < 1.5 * rs
        for fused in (False, True):
            rf = _dist_fp32(qi, qj, box, periodic, fused)
            err = np.abs(rf - r)[near].max()
            assert err <= bound, (box, far, fused, err, bound)
            # and it is not vacuous: the error reaches a sizeable part of it
            assert err > 0.01 * bound


def test_margin_keeps_pairs_that_fp32_alone_loses():
    """A pair at rc - 1e-6 near x = 900: FP32 alone puts it at or beyond rc,
    the widened radius keeps it."""
    rc = 1.0
    qi = np.array([[900.0, 2.0, 2.0]])
    qj = np.array([[900.0 + rc - 1e-6, 2.0, 2.0]])
    rf = _dist_fp32(qi, qj, (24.0, 8.0, 8.0), (0, 1, 1), False)[0]
    assert rf >= rc
    Q = 900.0 + rc
    assert rf < rc + 16.0 * U * (Q + rc)


def _min_image64(d, L):
    h = 0.5 * L
    return np.where(d > h, d - L, np.where(d < -h, d + L, d))


def test_displacement_bound_from_fp32_reference():
    """The list-build decision measures a particle's displacement from its
    build-time position kept in FP32 and widens it by 2^-23 (|x_f| + |y_f| +
    |z_f|) plus 2^-50 of the FP64 distance; the result must never fall below
    the true displacement from the exact FP64 position (the decision may only
    err towards an extra build).  Positions fill a periodic box (wrapped,
    some exactly at 0 or just below L, which FP32 may round up to L) and lie
    far outside a free boundary."""
    rng = np.random.default_rng(5)
    for box, periodic, spread in (([70.5, 70.5, 70.5], (1, 1, 1), 0.2),
                                  ([400.0, 20.0, 20.0], (0, 1, 1), 0.2),
                                  ([3.95, 3.95, 3.95], (1, 1, 1), 0.2)):
        box = np.asarray(box)
        n = 200000
        ref = rng.random((n, 3)) * box
        ref[:100] = 0.0
        ref[100:200] = np.nextafter(box, 0.0)
        if not periodic[0]:
            ref[200:400, 0] = rng.choice([-1.0, 1.0], 200) * rng.random(200) * 1e4
        move = (rng.random((n, 3)) - 0.5) * 2.0 * spread
        move[:1000] *= 1e-6  # displacements far below the FP32 rounding
        q = ref + move
        for k in range(3):
            if periodic[k]:
                q[:, k] = np.mod(q[:, k], box[k])
        rf = _f32(ref)
        d_true = np.zeros(n)
        d_comp = np.zeros((n, 3))
        for k in range(3):
            dt = q[:, k] - ref[:, k]
            dc = q[:, k] - rf[:, k].astype(np.float64)
            if periodic[k]:
                dt = _min_image64(dt, box[k])
                dc = _min_image64(dc, box[k])
            d_true += dt * dt
            d_comp[:, k] = dc
        d_true = np.sqrt(d_true)
        slack = 2.0 ** -23 * np.abs(rf.astype(np.float64)).sum(axis=1) + 2.0 ** -147
        bound = np.sqrt((d_comp * d_comp).sum(axis=1)) * (1.0 + 2.0 ** -50) + slack
        assert (bound >= d_true).all()
        # and the widening is small against any skin
        assert slack.max() < 1e-4 * max(1.0, np.abs(ref).max() / 100.0)


def test_block_quotient_from_fp32_reciprocal_is_exact():
    """The list build takes a cell's block coordinate c / B (B the block
    edge, 1 to 8) as trunc(fma(c, r, r / 2)) with r = 1/B rounded to FP32.
    The fused multiply-add rounds r (c + 1/2) once to FP32; for c below 2^21
    that product has at most 46 significant bits, so FP64 holds it exactly
    and one cast to FP32 reproduces the kernel's rounding.  Checked here for
    every c below 2^21, above the largest cell index the host admits."""
    c = np.arange(1 << 21, dtype=np.int64)
    for b in range(1, 9):
        r = np.float32(1.0) / np.float32(b)
        q = (np.float64(r) * (c.astype(np.float64) + 0.5)).astype(np.float32)
        assert (q.astype(np.int64) == c // b).all(), b
