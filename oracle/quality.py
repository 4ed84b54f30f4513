"""ORACLE of the distortion metrics -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this module; the product library never does.  Plain numpy in float64, written
from the definitions:

* Sec. 4.2 (evaluation metrics): distortion is measured by PSNR, and the
  bitrate is 32 bits divided by the compression ratio for fp32 data.
* The paper does not print the PSNR formula.  Reading: the form used with
  value-range-relative error bounds (Sec. 4.1), PSNR = 20 log10(vmax - vmin)
  - 10 log10(MSE), with vmin, vmax the range of the original field and MSE
  the mean of the squared pointwise differences.
* The maximum pointwise difference is the quantity the error bound of
  Sec. 2.3 limits.
* Each difference is (double)x - (double)y, one rounding to double; a
  position where x or y is NaN or infinite is counted, and then every metric
  is NaN.  mse == 0 gives PSNR +inf; a constant x with mse > 0 gives -inf.
"""
import math

import numpy as np


def quality(x, y):
    """Distortion of reconstruction ``y`` against original ``x`` (fp32 arrays
    of one shape).  Returns max_abs_err, mse, psnr, vmin, vmax, n, nonfinite."""
    x = np.ascontiguousarray(x, dtype=np.float32).ravel()
    y = np.ascontiguousarray(y, dtype=np.float32).ravel()
    if x.shape != y.shape:
        raise ValueError("shapes differ")
    n = int(x.size)
    finite = np.isfinite(x) & np.isfinite(y)
    nonfinite = int(n - np.count_nonzero(finite))
    if nonfinite:
        nan = float("nan")
        return {"max_abs_err": nan, "mse": nan, "psnr": nan, "vmin": nan, "vmax": nan, "n": n,
                "nonfinite": nonfinite}
    e = x.astype(np.float64) - y.astype(np.float64)
    mse = float(np.sum(e * e)) / n
    vmin, vmax = float(x.min()), float(x.max())
    rng = vmax - vmin
    if mse == 0.0:
        psnr = math.inf
    elif rng == 0.0:
        psnr = -math.inf
    else:
        psnr = 20.0 * math.log10(rng) - 10.0 * math.log10(mse)
    return {"max_abs_err": float(np.max(np.abs(e))), "mse": mse, "psnr": psnr, "vmin": vmin, "vmax": vmax,
            "n": n, "nonfinite": nonfinite}


def bitrate(ratio):
    """Average bits per fp32 value after compression (Sec. 4.2)."""
    return 32.0 / ratio


def overall_throughput(bw, ratio, t_compr):
    """Overall data-transfer throughput of Sec. 4.6: compression followed by
    moving the compressed bytes over a link of bandwidth ``bw``, in the units
    of ``bw`` and ``t_compr`` (input bytes per second):
    ((bw * ratio)^-1 + t_compr^-1)^-1."""
    return 1.0 / (1.0 / (bw * ratio) + 1.0 / t_compr)
