"""Round-to-nearest-even of float64 values to the storage formats, for the
codec tests (numpy only)."""
import numpy as np


def rne(x, fmt):
    """x (float64 array) rounded once, to nearest-even, to fmt ('f32', 'f16',
    'bf16'); returned as float64.  FP32 and FP16 use numpy's direct casts
    from double; BF16 (8 significant bits, FP32's exponent range) rounds the
    value to its spacing with round-half-even: 2^(e - 8) for |x| in
    [2^(e-1), 2^e), and the subnormal spacing 2^-133 below 2^-126."""
    x = np.asarray(x, dtype=np.float64)
    if fmt == "f32":
        return x.astype(np.float32).astype(np.float64)
    if fmt == "f16":
        return x.astype(np.float16).astype(np.float64)
    _, e = np.frexp(x)
    q = np.ldexp(1.0, np.maximum(e, -125) - 8)
    return np.rint(x / q) * q
