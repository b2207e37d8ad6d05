"""The FP64 FMA throughput probe of the benchmark's peak check (rok4e_fma_probe): bit-exact
against fused multiply-adds evaluated with exact rational arithmetic and one rounding."""
from fractions import Fraction

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def test_fma_probe_is_bit_exact():
    import torch
    from paper_1712_00953_amd import rok4e as R
    R.load()
    n, iters = 512, 3
    out = torch.empty(n, dtype=torch.float64, device="cuda:0")
    R.fma_probe(out, iters)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    b = 0.9999999999
    want = np.empty(n)
    for i in range(n):
        c = 1e-12 * float((i % 256) + 1)
        a = [1.0 + 0.125 * q for q in range(8)]
        for _ in range(iters):
            a = [_fma(x, b, c) for x in a]
        want[i] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]))
    np.testing.assert_array_equal(got, want)
    with pytest.raises(R.Rok4eError):
        R.fma_probe(out[:100], iters)
