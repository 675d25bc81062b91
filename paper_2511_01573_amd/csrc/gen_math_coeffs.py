"""Generates the polynomial coefficients of gm_math.hpp (run by hand; output
pasted into the header).

exp:  e^r on [-ln2/2, ln2/2], degree 11, Chebyshev approximation (mpmath
      chebyfit, 50 digits) -- max error 3.2e-18.
cos:  cos(r) = C(z), z = r^2, z in [0, (pi/2)^2], degree 9 in z -- 6.4e-21
      (reduction by pi, |r| <= pi/2).
sin:  sin(r) = r (1 + z Q(z)), Q(z) = (sin(sqrt z)/sqrt z - 1)/z, z in
      [0, (pi/2)^2], degree 8 in z -- 5.0e-22 (same reduction).
Coefficients are printed as hexadecimal doubles, highest degree first.
"""
import mpmath as mp

mp.mp.dps = 50


def fit(f, a, b, deg):
    poly, err = mp.chebyfit(f, [a, b], deg + 1, error=True)
    return [float(c) for c in poly], err


def show(name, coeffs, err):
    print(f"// {name}: max |error| {mp.nstr(err, 3)}")
    print(f"constexpr double {name}[{len(coeffs)}] = {{")
    print(",\n".join(f"    {c.hex()}" for c in coeffs) + "};")


ln2 = mp.log(2)
show("kExpPoly", *fit(mp.exp, -ln2 / 2, ln2 / 2, 11))
show("kCosPoly", *fit(lambda z: mp.cos(mp.sqrt(z)) if z > 0 else mp.mpf(1), 0, (mp.pi / 2) ** 2, 9))


def sin_q(z):
    if z == 0:
        return mp.mpf(-1) / 6
    r = mp.sqrt(z)
    return (mp.sin(r) / r - 1) / z


show("kSinPoly", *fit(sin_q, 0, (mp.pi / 2) ** 2, 8))
# Cody-Waite constants
l2hi = float(ln2)
l2lo = float(ln2 - mp.mpf(l2hi))
print("constexpr double kLn2Hi =", l2hi.hex(), ";")
print("constexpr double kLn2Lo =", l2lo.hex(), ";")
print("constexpr double kInvLn2 =", float(1 / ln2).hex(), ";")
p1 = float(mp.pi)
p2 = float(mp.pi - mp.mpf(p1))
p3 = float(mp.pi - mp.mpf(p1) - mp.mpf(p2))
print("constexpr double kPi_1 =", p1.hex(), ";")
print("constexpr double kPi_2 =", p2.hex(), ";")
print("constexpr double kPi_3 =", p3.hex(), ";")
print("constexpr double kInvPi =", float(1 / mp.pi).hex(), ";")
