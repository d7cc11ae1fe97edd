"""Writes segment_example.json: the colour-segment worked example of the
oracle pins, evaluated in closed form with 40-digit decimal arithmetic.

A pixel on the segment between two LR colours, I_p = t L_a + (1 - t) L_b,
with l = ||L_a - L_b||:
  Eq. 4 (Sec. 3.1):  alpha = ((I_p - L_b).(L_a - L_b)) / (l^2 + eps) = t l^2 / (l^2 + eps)
  Eq. 5 (Sec. 3.2, anchor L_a, the nearest colour when t > 1/2):
                     alpha = ||I_p - L_b|| / (||I_p - L_a|| + ||I_p - L_b|| + eps) = t l / (l + eps)
  and in both cases the reconstruction lies on the segment, so the error is
  |t - alpha| l.  With eps = 0 both weights are t and the error is 0.

Nothing here calls the oracle or the HIP library: the values are the closed
forms above.  Run from the repository root:

    python tests/golden/make_segment_example.py [--check]

``--check`` compares with the committed file instead of writing it.
"""
import decimal
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "segment_example.json")

D = decimal.Decimal


def values():
    ctx = decimal.Context(prec=40)
    La = [D(1), D(0), D(0)]
    Lb = [D(0), D(0), D(1)]
    t = D("0.75")
    eps = D("0.001")
    l2 = ctx.add(ctx.add(ctx.power(La[0] - Lb[0], 2), ctx.power(La[1] - Lb[1], 2)), ctx.power(La[2] - Lb[2], 2))
    l = ctx.sqrt(l2)
    Ip = [ctx.add(ctx.multiply(t, a), ctx.multiply(1 - t, b)) for a, b in zip(La, Lb)]
    eq4_alpha = ctx.divide(ctx.multiply(t, l2), ctx.add(l2, eps))
    eq4_err = ctx.multiply(ctx.subtract(t, eq4_alpha), l)
    eq5_alpha = ctx.divide(ctx.multiply(t, l), ctx.add(l, eps))
    eq5_err = ctx.multiply(ctx.subtract(t, eq5_alpha), l)
    return dict(La=La, Lb=Lb, t=t, Ip=Ip, eps=eps, eq4_alpha=eq4_alpha, eq4_err=eq4_err,
                eq5_alpha=eq5_alpha, eq5_err=eq5_err)


def _vec(v):
    return "[" + ", ".join("%.1f" % float(x) if x == x.to_integral_value() else str(x) for x in v) + "]"


def text():
    v = values()
    head = {
        "what": "A pixel on the colour segment between two LR colours, window holding only those two colours",
        "cite": "Sec. 3.1 Eq. 4 (projection weight with eps = 1e-3); Sec. 3.2 Eq. 5 (fast weight) and Algorithm 1 "
                "(anchor = most similar colour)",
        "derivation": "I_p = t L_a + (1 - t) L_b with L_a = (1,0,0), L_b = (0,0,1), l = ||L_a - L_b|| = sqrt(2), "
                      "t = 0.75. Eq. 4: alpha = ((I_p - L_b).(L_a - L_b)) / (l^2 + eps) = t l^2 / (l^2 + eps); "
                      "error = (t - alpha) l. Eq. 5 with the anchor L_a (nearest colour since t > 1/2): alpha = "
                      "||I_p - L_b|| / (||I_p - L_a|| + ||I_p - L_b|| + eps) = t l / (l + eps); error = (t - alpha) l. "
                      "With eps = 0 both give alpha = t and zero error (Sec. 3.2 states Eq. 4 reduces to Eq. 5 on the "
                      "colour line). Values evaluated with 40-digit decimal arithmetic.",
    }
    lines = ["{"]
    for key, val in head.items():
        lines.append("  %s: %s," % (json.dumps(key), json.dumps(val)))
    lines.append('  "L_a": %s,' % _vec(v["La"]))
    lines.append('  "L_b": %s,' % _vec(v["Lb"]))
    lines.append('  "t": %s,' % v["t"])
    lines.append('  "I_p": %s,' % _vec(v["Ip"]))
    lines.append('  "eps": %s,' % v["eps"])
    for key in ("eq4_alpha", "eq4_err", "eq5_alpha", "eq5_err"):
        lines.append('  "%s": %s,' % (key, v[key]))
    lines.append('  "eps0_alpha": %s,' % v["t"])
    lines.append('  "eps0_err": 0.0')
    lines.append("}")
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    new = text()
    if "--check" in sys.argv:
        old = open(OUT).read()
        if json.loads(old, parse_float=D) != json.loads(new, parse_float=D):
            sys.exit("segment_example.json differs from the closed forms")
        print("segment_example.json matches the closed forms")
    else:
        with open(OUT, "w") as f:
            f.write(new)
        print("wrote", OUT)
