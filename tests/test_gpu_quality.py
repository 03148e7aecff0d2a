"""The sampler on the GPU recovers the small four-cluster recipe from one
cluster (split-BF16, split/merge moves only): adjusted Rand index above 0.95
and four clusters after 40 iterations.  The paper's own quality figures use
data that is not available, so this is a sanity check, not a parity pin."""
import sys

import pytest

from paper_1812_10048_amd import quality

pytestmark = pytest.mark.gpu


def test_small_recipe_recovered_from_one_cluster():
    print("quality c1", flush=True)
    sys.stdout.flush()
    recs = quality.run("c1", iters=40, alpha=1.0, precision="split_bf16", seed=0, every=10, k_max=64,
                       split_q=False, new_cluster=False)
    last = recs[-1]
    assert last["ari"] > 0.95 and last["K"] == 4, last
