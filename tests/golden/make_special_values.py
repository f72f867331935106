"""Writes special_values.txt: exact a_l0 of a unit-weight point at the north pole,
the south pole and the equator, for l <= 64, from closed forms only (no oracle,
no GPU code):

* north pole, theta = 0: P_l(1) = 1 (the normalisation the paper uses in Sec. 2.1),
  so a_l0 = sqrt((2l+1)/4pi) and a_lm = 0 for m > 0;
* south pole, theta = pi: reflection in x costs (-1)^(l-m) (App. A.1), so
  a_l0 = (-1)^l sqrt((2l+1)/4pi);
* equator, theta = pi/2: P_l(0) = (-1)^(l/2) (l-1)!!/l!! for even l, 0 for odd l
  (textbook value of the Legendre polynomial at 0).

Values are evaluated with exact rationals, then one square root in 50-digit
decimal, and written with 20 significant digits.  Run: python make_special_values.py
"""
import decimal
import os
from fractions import Fraction

decimal.getcontext().prec = 50
PI = decimal.Decimal("3.14159265358979323846264338327950288419716939937510")
LMAX = 64


def legendre_at_zero(l: int) -> Fraction:
    if l % 2:
        return Fraction(0)
    num = 1
    den = 1
    for k in range(1, l, 2):
        num *= k
    for k in range(2, l + 1, 2):
        den *= k
    return Fraction((-1) ** (l // 2) * num, den)


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "special_values.txt")
    lines = ["# l  theta_label  a_l0 (unit weight, phi arbitrary; a_lm = 0 for m > 0 at the poles)",
             "# north: P_l(1)=1 (Sec. 2.1); south: reflection phase (-1)^(l-m) (App. A.1);",
             "# equator: P_l(0) = (-1)^(l/2) (l-1)!!/l!!, l even; written by make_special_values.py"]
    for l in range(LMAX + 1):
        norm = (decimal.Decimal(2 * l + 1) / (4 * PI)).sqrt()
        p0 = legendre_at_zero(l)
        vals = {"north": norm, "south": norm * (-1 if l % 2 else 1),
                "equator": norm * decimal.Decimal(p0.numerator) / decimal.Decimal(p0.denominator)}
        for lab in ("north", "south", "equator"):
            lines.append(f"{l} {lab} {vals[lab]:.20e}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out)


if __name__ == "__main__":
    main()
