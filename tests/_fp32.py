"""Single-precision error bounds of the energy and its gradients (Eq. 1 and
its derivatives), for tests that grade the FP32 kernels against the
double-precision oracle element by element.

The kernels read FP32 spins and constants and form every site's field sum,
dot products and anisotropy terms with FP32 fused multiply-adds (unit
roundoff u32 = 2^-24); the sums over sites and over groups of
configurations are in double.  With s_i = sum_j |J_ij| + |B| + 2 |k_i| (unit
spins), the bounds below allow one rounding per term of each FP32 chain,
twice over when the oracle's inputs are not rounded to FP32 first, plus the
final rounding of an FP32 result:

  dE/dS_i (weight w)        (2 deg_i + 8) u32 s_i w
  dE/dJ_b (weights w_c)     (4 + G) u32 sum_c w_c      G: configurations summed in FP32
  dE/dk_i                   (8 + G) u32 sum_c w_c
  dE/dB                     8 u32 n sum_c w_c
"""
import numpy as np

U32 = 2.0 ** -24


def site_scale(lat, B):
    """s_i for unit spins."""
    rows = np.repeat(np.arange(lat.n), np.diff(lat.row_ptr))
    s = np.zeros(lat.n)
    np.add.at(s, rows, np.abs(lat.J))
    k = np.zeros(lat.n) if lat.k is None else np.abs(lat.k)
    return s + abs(B) + 2.0 * k


def grad_bounds(lat, B, w, G=32):
    """Per-element bounds: (dS [n] per unit weight, dJ, dk, dB) for weights w."""
    deg = np.diff(lat.row_ptr)
    sw = float(np.sum(np.abs(w)))
    g = min(G, int(np.count_nonzero(w)))
    dS = (2 * deg + 8) * U32 * site_scale(lat, B)
    return dS, (4 + g) * U32 * sw, (8 + g) * U32 * sw, 8 * U32 * lat.n * sw
