"""Round-to-nearest-even onto the BF16 and OCP FP8-e4m3 value grids (oracle).

Written from the formats' definitions, on float64 inputs:

* BF16: 1 sign, 8 exponent, 7 stored mantissa bits (8 significant bits), the
  exponent range of FP32.  A finite x = m 2^e with 0.5 <= |m| < 1 rounds to
  rint(m 2^8) 2^(e-8); rint is round-half-even.  Values below the smallest
  normal 2^-126 use the fixed subnormal step 2^-133.
* E4M3 (OCP 8-bit float, the format gfx950's FP8 MFMA reads): 4 exponent bits
  with bias 7, 3 mantissa bits, no infinities, largest finite value
  448 = 1.75 * 2^8, smallest normal 2^-6 and subnormal step 2^-9.  Rounding is
  to nearest even and saturates at +-448.

Pins (tests/test_oracle_post.py): torch's own float -> bfloat16 and
float -> float8_e4m3fn casts on exactly representable float32 inputs, the
format's listed extreme values (tests/golden/e4m3_points.txt), and
hand-checked ties (tests/test_oracle_quant_points.py).
"""
import numpy as np


def _round_sig(x, sig_bits, min_exp, step_exp):
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                       # x = m 2^e, 0.5 <= |m| < 1
    normal = np.ldexp(np.rint(np.ldexp(m, sig_bits)), e - sig_bits)
    sub = np.ldexp(np.rint(np.ldexp(x, -step_exp)), step_exp)
    return np.where(np.abs(x) >= np.ldexp(1.0, min_exp), normal, sub)


def bf16_round(x):
    """Nearest BF16 value (ties to even), as float64."""
    return _round_sig(x, 8, -126, -133)


E4M3_MAX = 448.0


def e4m3_round(x):
    """Nearest OCP E4M3 value (ties to even, saturating at +-448), as float64."""
    r = _round_sig(x, 4, -6, -9)
    return np.clip(r, -E4M3_MAX, E4M3_MAX)
