"""Writes the hand-derivation fixtures of this folder with exact rational arithmetic.

Nothing here calls the library under test or the oracle: every value is an
exact rational (``fractions.Fraction``) rounded to binary32 or kept exact, by
the rules stated next to each step, so that every printed line can be checked
by hand.  Run ``python tests/golden/derive.py`` to rewrite

* ``eq1_lambda001.txt`` -- Eq. 1 (Sec. II.C.3) at lambda = 0.01, evaluated in
  binary32 in the order fixed for the filter:
      fr(x) = fl32(lambda * x),  a = fl32(fr(r) - fr(i)),  b = fl32(fr(c) - fr(j)),
      e = fl32(I_q - I_p),  d = fl32(e*e + fl32(b*b + fl32(a*a)))
  (the two outer roundings are those of fused multiply-adds: the product is
  not rounded on its own);
* ``coupling_3class.txt`` -- the pairwise coupling of Sec. II.C.1 (the second
  method of Wu, Lin and Weng that the paper cites) for three classes, sweep by
  sweep, with the stopping rule max_t |(Qp)_t - p'Qp| < eps.
"""
from __future__ import annotations

import os
from fractions import Fraction as F

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# IEEE 754 binary32, round to nearest, ties to even (normal numbers only:
# every value below stays far above 2^-126).
# ---------------------------------------------------------------------------
def binade(x: F) -> int:
    """The exponent k with 2^k <= x < 2^(k+1), x > 0."""
    k = x.numerator.bit_length() - x.denominator.bit_length()
    if F(2) ** k > x:
        k -= 1
    if F(2) ** (k + 1) <= x:
        k += 1
    return k


def rne32(x: F) -> F:
    if x == 0:
        return F(0)
    sign = -1 if x < 0 else 1
    m = abs(x)
    k = binade(m)
    if k < -126:
        raise ValueError("subnormal result: choose another case")
    ulp = F(2) ** (k - 23)
    q = m / ulp
    n = q.numerator // q.denominator
    rest = q - n
    if rest > F(1, 2) or (rest == F(1, 2) and n % 2 == 1):
        n += 1
    return sign * n * ulp


def hexf(x: F) -> str:
    """Exact hexadecimal form of a dyadic rational, e.g. -0x1.8p-3."""
    if x == 0:
        return "0x0p+0"
    if x.denominator & (x.denominator - 1):
        raise ValueError("not dyadic")
    sign = "-" if x < 0 else ""
    m = abs(x)
    k = binade(m)
    frac = m / F(2) ** k - 1          # in [0, 1), dyadic
    digits = ""
    while frac:
        frac *= 16
        d = frac.numerator // frac.denominator
        digits += "0123456789abcdef"[d]
        frac -= d
    return f"{sign}0x1{'.' + digits if digits else ''}p{k:+d}"


def f32bits(x: F) -> int:
    """Bit pattern of a positive normal binary32 value."""
    k = binade(x)
    mant = x / F(2) ** k * 2 ** 23
    assert mant.denominator == 1
    return ((k + 127) << 23) | (int(mant) - (1 << 23))


# ---------------------------------------------------------------------------
# Eq. 1 at lambda = 0.01
# ---------------------------------------------------------------------------
LAMBDA = rne32(F(1, 100))  # the binary32 nearest to 0.01

# (r, c, I_q, i, j, I_p): query pixel (r, c) and candidate (i, j) with their
# one-band values (binary32, written exactly).  Chosen so that every
# alternative evaluation order listed in the file changes the result's bits.
EQ1_CASES = [
    (20, 20, "0x1.a558f2p-1", 17, 14, "0x1.b9a15ap-1"),
    (7, 301, "0x1.3c9f1ep-2", 10, 298, "0x1.3a1b06p-2"),
    (31, 296, "0x1.bfd73cp-5", 34, 297, "0x1.11483ap-4"),
    (2, 88, "0x1.02c6f4p-3", 0, 85, "0x1.1f0a5ep-3"),
    (15, 56, "0x1.302df8p-1", 13, 54, "0x1.32b9p-1"),
    (12, 395, "0x1.22d27ep-1", 11, 401, "0x1.36c6dep-1"),
    (38, 5, "0x1.2d9ee8p-4", 35, 0, "0x1.51c63ap-4"),
]


def eq1_lines():
    out = [
        "# Eq. 1 (Sec. II.C.3) at lambda = 0.01 in binary32, derived by hand with exact",
        "# rationals; every rounding is to nearest, ties to even.  Written by derive.py.",
        "#",
        "#   fr(x) = fl32(lambda * x)      a = fl32(fr(r) - fr(i))     b = fl32(fr(c) - fr(j))",
        "#   e = fl32(I_q - I_p)           h = fl32(a * a)",
        "#   t = fl32(b * b + h)  (fused)  d = fl32(e * e + t)  (fused)",
        "#",
        f"# lambda = fl32(0.01) = {hexf(LAMBDA)} = {LAMBDA.numerator}/{LAMBDA.denominator}",
        "#",
        "# Format: r c I_q i j I_p : d d_bits   (query (r, c), candidate (i, j))",
    ]
    for r, c, iq, i, j, ip in EQ1_CASES:
        Iq, Ip = F(float.fromhex(iq)), F(float.fromhex(ip))
        assert rne32(Iq) == Iq and rne32(Ip) == Ip
        fr_r, fr_i = rne32(LAMBDA * r), rne32(LAMBDA * i)
        fr_c, fr_j = rne32(LAMBDA * c), rne32(LAMBDA * j)
        a = rne32(fr_r - fr_i)
        b = rne32(fr_c - fr_j)
        e = rne32(Iq - Ip)
        h = rne32(a * a)
        t = rne32(b * b + h)
        d = rne32(e * e + t)
        out += [
            "#",
            f"# query ({r}, {c}), I_q = {iq}; candidate ({i}, {j}), I_p = {ip}",
            f"#   lambda*{r} = {hexf(LAMBDA * r)} -> fr({r}) = {hexf(fr_r)}",
            f"#   lambda*{i} = {hexf(LAMBDA * i)} -> fr({i}) = {hexf(fr_i)}",
            f"#   lambda*{c} = {hexf(LAMBDA * c)} -> fr({c}) = {hexf(fr_c)}",
            f"#   lambda*{j} = {hexf(LAMBDA * j)} -> fr({j}) = {hexf(fr_j)}",
            f"#   fr({r}) - fr({i}) = {hexf(fr_r - fr_i)} -> a = {hexf(a)}",
            f"#   fr({c}) - fr({j}) = {hexf(fr_c - fr_j)} -> b = {hexf(b)}",
            f"#   I_q - I_p = {hexf(Iq - Ip)} -> e = {hexf(e)}",
            f"#   a*a = {hexf(a * a)} -> h = {hexf(h)}",
            f"#   b*b + h = {hexf(b * b + h)} -> t = {hexf(t)}",
            f"#   e*e + t = {hexf(e * e + t)} -> d = {hexf(d)}",
            f"{r} {c} {iq} {i} {j} {ip} : {hexf(d)} 0x{f32bits(d):08x}",
        ]
    return out


# ---------------------------------------------------------------------------
# Pairwise coupling, three classes
# ---------------------------------------------------------------------------
# r_ij for the pairs (0,1), (0,2), (1,2); r_ji = 1 - r_ij.
COUPLING_CASES = [
    (F(1, 10), F(3, 5), F(3, 4)),
    (F(9, 10), F(1, 20), F(3, 4)),
]


def couple_exact(r01, r02, r12, eps, max_sweeps=100):
    C = 3
    R = [[F(0)] * C for _ in range(C)]
    R[0][1], R[0][2], R[1][2] = r01, r02, r12
    R[1][0], R[2][0], R[2][1] = 1 - r01, 1 - r02, 1 - r12
    Q = [[F(0)] * C for _ in range(C)]
    for t in range(C):
        for j in range(C):
            Q[t][j] = (sum(R[s][t] ** 2 for s in range(C) if s != t) if j == t
                       else -R[j][t] * R[t][j])
    p = [F(1, C)] * C
    log = []
    sweeps = 0
    for _ in range(max_sweeps):
        Qp = [sum(Q[t][j] * p[j] for j in range(C)) for t in range(C)]
        pQp = sum(p[t] * Qp[t] for t in range(C))
        res = max(abs(Qp[t] - pQp) for t in range(C))
        log.append((sweeps, list(p), res))
        if res < eps:
            break
        for t in range(C):
            Qp = [sum(Q[u][j] * p[j] for j in range(C)) for u in range(C)]
            pQp = sum(p[u] * Qp[u] for u in range(C))
            off = sum(Q[t][j] * p[j] for j in range(C) if j != t)
            q = list(p)
            q[t] = (pQp - off) / Q[t][t]
            s = sum(q)
            p = [x / s for x in q]
        sweeps += 1
    return Q, p, sweeps, log


def dec(x: F, digits: int = 22) -> str:
    return f"{float(x):.17g}" if digits <= 17 else _dec(x, digits)


def _dec(x: F, digits: int) -> str:
    sign = "-" if x < 0 else ""
    x = abs(x)
    scaled = x * 10 ** digits
    n = (scaled.numerator * 2 + scaled.denominator) // (2 * scaled.denominator)
    s = str(n).rjust(digits + 1, "0")
    return f"{sign}{s[:-digits]}.{s[-digits:]}"


def coupling_lines():
    out = [
        "# Pairwise coupling (Sec. II.C.1; second method of Wu, Lin and Weng), three",
        "# classes, derived with exact rationals.  Written by derive.py.",
        "#",
        "#   Q[t][t] = sum_{s != t} r_st^2,  Q[t][j] = -r_jt r_tj",
        "#   p = (1/3, 1/3, 1/3); each sweep updates t = 0, 1, 2 in turn:",
        "#     p[t] <- (p'Qp - sum_{j != t} Q[t][j] p[j]) / Q[t][t], then p <- p / sum(p)",
        "#   a sweep starts only while max_t |(Qp)_t - p'Qp| >= eps",
        "#",
        "# Format: case r01 r02 r12 | stop eps sweeps p0 p1 p2   (decimals to 22 places)",
    ]
    for r01, r02, r12 in COUPLING_CASES:
        out.append("#")
        out.append(f"# r01 = {r01}, r02 = {r02}, r12 = {r12}")
        for eps_label, eps in (("0.005/3", F(5, 3000)), ("0.005", F(5, 1000))):
            Q, p, sweeps, log = couple_exact(r01, r02, r12, eps)
            if eps_label == "0.005/3":
                out.append("#   Q = " + "; ".join(" ".join(str(v) for v in row) for row in Q))
            for k, pk, res in log:
                out.append(f"#   eps {eps_label}: start of sweep {k + 1}: p = "
                           f"({', '.join(_dec(v, 12) for v in pk)}), residual {_dec(res, 12)}"
                           + ("  < eps: stop" if res < eps else ""))
            out.append(f"{r01} {r02} {r12} | {eps_label} {sweeps} "
                       + " ".join(_dec(v, 22) for v in p))
    return out


def main():
    with open(os.path.join(HERE, "eq1_lambda001.txt"), "w") as f:
        f.write("\n".join(eq1_lines()) + "\n")
    with open(os.path.join(HERE, "coupling_3class.txt"), "w") as f:
        f.write("\n".join(coupling_lines()) + "\n")


if __name__ == "__main__":
    main()
