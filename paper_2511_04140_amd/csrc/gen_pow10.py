"""Prints the fl(10^k) tables embedded in codec_device.hpp.

Each entry is the binary64 (binary32) value nearest to the exact rational
10^k (ties to even), rounded directly from the rational with integer
arithmetic, so no intermediate rounding is involved.
Run: python gen_pow10.py
"""
from fractions import Fraction


def round_to_binary(q: Fraction, mant_bits: int) -> Fraction:
    """Nearest value with mant_bits+1 significant bits (ties to even)."""
    e = q.numerator.bit_length() - q.denominator.bit_length()
    while Fraction(2) ** e > q:
        e -= 1
    while Fraction(2) ** (e + 1) <= q:
        e += 1
    scale = Fraction(2) ** (mant_bits - e)
    m = q * scale
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return Fraction(fl) / scale


def hexf(q: Fraction, mant_bits: int) -> str:
    v = round_to_binary(q, mant_bits)
    e = v.numerator.bit_length() - v.denominator.bit_length()
    while Fraction(2) ** e > v:
        e -= 1
    while Fraction(2) ** (e + 1) <= v:
        e += 1
    m = v / Fraction(2) ** e           # in [1, 2)
    frac = (m - 1) * (1 << mant_bits)
    assert frac.denominator == 1
    digits = (mant_bits + 3) // 4
    frac_int = int(frac) << (4 * digits - mant_bits)
    return f"0x1.{frac_int:0{digits}x}p{e:+d}"


if __name__ == "__main__":
    print("// k = -22..22, binary64")
    print(",\n".join(hexf(Fraction(10) ** k, 52) for k in range(-22, 23)))
    print("// k = -10..10, binary32")
    print(",\n".join(hexf(Fraction(10) ** k, 23) + "f" for k in range(-10, 11)))
