"""The matrix-core form of the list build's int16 pair test, checked on the
CPU: the 16 f16 slots of a candidate and a home atom are exact in f16, and
their products accumulated in f32 in any order give exactly 1/2 - S, where
S = q_i.(2 q'_j) + C_j - B_i is the integer the vector form tests (S > 0:
the pair survives).  Ranges are the extremes the kernel admits: |q| <= 127,
shifted offsets q' = q + 250 o with |o| <= 2 (half-size subcells), d <= 10,
C = T_j - |q'_j|^2 with T up to the half-grid share bound, B = |q_i|^2 - T_i.
This pins the encoding's arithmetic, not the kernel (which the GPU list
tests compare with the definition)."""
import numpy as np
import pytest


def cand_slots(q2, C, d):
    """Slots of a candidate: [2q'_0 .. 2q'_{d-1}, 2048, 1, 1, floor(C/2048), C mod 2048, 0 ..]."""
    C = max(C, -4194304)  # an empty lane
    s = np.zeros(16, dtype=np.int64)
    s[:d] = q2
    s[d:d + 5] = [2048, 1, 1, C >> 11, C & 2047]
    return s


def home_slots(q, B, d):
    """Slots of a home atom: [-q_0 .. -q_{d-1}, floor(B/2048), B mod 2048, 1/2, -2048, -1, 0 ..]."""
    s = np.zeros(16, dtype=np.float64)
    s[:d] = -q
    s[d:d + 5] = [B >> 11, B & 2047, 0.5, -2048, -1]
    return s


@pytest.mark.parametrize("d", [2, 6, 10])
def test_slots_exact_and_sum_exact_in_any_order(d):
    g = np.random.default_rng(100 + d)
    Tmax = 2 * (250 + np.sqrt(d) / 2) ** 2 + 1   # the half-grid share bound
    for _ in range(400):
        q = g.integers(-127, 128, d)
        o = g.integers(-2, 3, d)
        qp = g.integers(-127, 128, d) + 250 * o
        Ti, Tj = (int(g.integers(1, Tmax)) for _ in range(2))
        if g.random() < 0.3:  # extremes
            q = g.choice([-127, 127], d)
            qp = g.choice([-627, 627], d)
            Ti = Tj = int(Tmax)
        B = int(q @ q) - Ti
        C = Tj - int(qp @ qp)
        a = cand_slots(2 * qp, C, d).astype(np.float64)
        b = home_slots(q, B, d)
        # every slot exact in f16
        assert np.array_equal(a.astype(np.float16).astype(np.float64), a)
        assert np.array_equal(b.astype(np.float16).astype(np.float64), b)
        S = int(q @ (2 * qp)) + C - B
        want = 0.5 - S
        prods = (a * b).astype(np.float32)   # each product exact in f32
        assert np.array_equal(prods.astype(np.float64), a * b)
        for _ in range(4):  # f32 accumulation in several orders
            acc = np.float32(0.0)
            for p in prods[g.permutation(16)]:
                acc = np.float32(acc + p)
            assert float(acc) == want
        assert (want < 0) == (S > 0)


def test_empty_lane_never_passes():
    """An empty lane's C becomes -2^22, and S stays negative for every home atom."""
    d = 10
    q = np.full(d, 127)
    qp = np.full(d, 627)
    Ti = int(2 * (250 + np.sqrt(d) / 2) ** 2 + 1)
    B = int(q @ q) - Ti
    a = cand_slots(2 * qp, -0x3fffffff, d).astype(np.float64)
    b = home_slots(q, B, d)  # q_i.(2 q'_j) at its largest
    assert float(a @ b) > 0  # 1/2 - S > 0: the pair fails
