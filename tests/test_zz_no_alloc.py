"""gsgp_reconstruct_static, the reconstruction entry point that uses the
library's own device scratch array instead of caller scratch: through the C
ABI, its output equals gsgp_reconstruct's bit for bit on two calls in a row
(the second on a smaller input, so that it reads the array after a larger
call left it full), it equals the oracle's reconstruction along the same
lineage, and a reconstruction larger than the array is refused before any
device work."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2106_04034_amd import gsgp
from tests.gpu_helpers import dataset, oracle_config, rel_err

pytestmark = pytest.mark.gpu


def test_static_scratch_reconstruction_equals_the_scratch_argument_form():
    d = dataset(700, 300, 6, seed=21)
    G = 10
    s = gsgp.Settings(pop_size=48, pool_size=32, n_generations_max=G, seed=23)
    R = gsgp.Runner(s, [d])
    R.eval_population()
    R.generation(G, stats=False)
    res = orc.run(oracle_config(s), d.X_train, d.y_train, d.X_test, d.y_test, G)
    best = int(R.stats(0, G, 1)[0]["best_index"])
    rng = np.random.default_rng(77)
    X1 = rng.uniform(-1.0, 1.0, size=(5000, 6))
    X2 = rng.uniform(-1.0, 1.0, size=(130, 6))
    for gen, i, X in ((G, best, X1), (G - 3, 5, X2)):
        print(f"reconstruct_static: gen {gen}, individual {i}, {X.shape[0]} cases", flush=True)
        want = R.reconstruct(0, gen, i, X)
        got = R.reconstruct_static(0, gen, i, X)
        assert np.array_equal(got, want), (gen, i)
        assert rel_err(got, orc.reconstruct(res, oracle_config(s), gen, i, X), 1.0) <= 1e-12
    # a reconstruction beyond the array is refused with a clear error
    size = ctypes.c_size_t(0)
    n_big = 1_200_000
    gsgp.check(gsgp.lib().gsgp_reconstruct_scratch_size(R._h, 0, G, best, n_big, ctypes.byref(size)), "size")
    assert size.value > (64 << 20)
    Xbig = np.zeros((n_big, 6))
    with pytest.raises(gsgp.GSGPError) as e:
        R.reconstruct_static(0, G, best, Xbig)
    assert e.value.status == -3 and "static scratch" in str(e.value)
    # the handle still works after the refusal
    assert np.array_equal(R.reconstruct_static(0, G, best, X2), R.reconstruct(0, G, best, X2))
    R.close()
