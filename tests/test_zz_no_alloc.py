"""GPU test of pt_reciprocal_estimate_noalloc, the table-mode reciprocal estimator that allocates
nothing: on two calls in a row (the second with a shorter table, so the fixed device array still
holds the first call's longer cumulative sums), its estimates and sample counts equal those of
pt_reciprocal_estimate on the same query bit for bit (the same kernels on the same inputs), and
their mean is 1 / sum f within 4 standard errors. Tables beyond the limit are rejected."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_table_matches_allocating_entry_point():
    import torch
    from paper_2503_23412_amd import pt
    pt.lib()
    rng = np.random.Generator(np.random.Philox(key=77))
    n_est = 1 << 18
    for n, seed in ((200_000, 3), (1_000, 4)):
        f = rng.uniform(0.0, 1.0, n)
        q = rng.uniform(0.2, 1.0, n)
        q /= q.sum()
        B = 1.5 * float((f / q).max())
        fd = torch.tensor(f, dtype=torch.float32, device="cuda")
        qd = torch.tensor(q, dtype=torch.float32, device="cuda")
        a = torch.empty(n_est, device="cuda")
        na = torch.empty(n_est, dtype=torch.int32, device="cuda")
        b = torch.empty(n_est, device="cuda")
        nb = torch.empty(n_est, dtype=torch.int32, device="cuda")
        pt.reciprocal_table(fd, qd, B, n_est, a, na, seed=seed)
        pt.reciprocal_table_noalloc(fd, qd, B, n_est, b, nb, seed=seed)
        torch.cuda.synchronize()
        print(f"noalloc n={n}: mean {float(b.double().mean()):.6g} target {1 / f.sum():.6g}", flush=True)
        assert torch.equal(na, nb)
        assert torch.equal(a, b)
        nsv = nb.cpu().numpy().astype(np.int64)
        assert (nsv >> 31 & 1).sum() == 0
        est = b.double().cpu().numpy()
        assert abs(est.mean() - 1 / f.sum()) < 4 * est.std() / math.sqrt(n_est)
    big = torch.ones(pt.NOALLOC_TABLE_MAX + 1, device="cuda")
    out = torch.empty(4, device="cuda")
    ns = torch.empty(4, dtype=torch.int32, device="cuda")
    with pytest.raises(pt.PTError) as e:
        pt.reciprocal_table_noalloc(big, big / big.numel(), 2.0, 4, out, ns)
    assert e.value.code == -1
