"""The adaptive duplicate-vs-partition policy driving real Jacobi sweeps on
the device: the field is bit-exact against the oracle whatever modes were
taken, and the library's decisions equal the oracle policy replayed on the
same measured step times."""
import numpy as np
import pytest

import oracle
from oracle import adapt as A
from paper_2110_14340_amd import adaptive, inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,n,steps,peak", [((514, 514), 4, 24, 153e9), ((2050, 1026), 8, 30, 1e15)])
def test_adaptive_jacobi_bit_exact_and_policy_parity(shape, n, steps, peak):
    print(f"adaptive jacobi {shape} n={n} steps={steps}", flush=True)
    u0 = inputs.jacobi_grid(*shape, seed=3)
    out, modes, times = adaptive.jacobi_adaptive(u0, steps, n, peak)
    assert np.array_equal(out, oracle.jacobi2d(u0, steps))
    ws = 8.0 * (shape[0] - 2) * (shape[1] - 2)
    assert modes == A.run([(t, 0.0, ws) for t in times], n, peak)
    assert all(t > 0 for t in times)
