"""The allocation-free interpolation entry point (tsm_prolong_noalloc)
against tsm_prolong through the C ABI: bitwise equal on two calls in a row
on one device, the second with a smaller batch (the static workspace keeps
the first call's contents), and its size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(rng, n):
    lo = rng.choice(np.array([2, 5, 8, 16, 31, 32], np.int32), n)
    ln = np.where(rng.uniform(size=n) < 0.5, 2 * lo, lo).astype(np.int32)
    return lo, ln


def test_noalloc_prolong_matches_allocating_entry_point():
    import torch
    from paper_2103_17040_amd import tsm
    rng = np.random.default_rng(17)
    for n in (3000, 257):           # the second call is smaller
        lo, ln = _case(rng, n)
        n_old = int(((lo.astype(np.int64) + 1) ** 2).sum())
        n_new = int(((ln.astype(np.int64) + 1) ** 2).sum())
        print(f"[gpu-case] prolong_noalloc n_inst={n} n_old={n_old} n_new={n_new}", flush=True)
        vo = torch.tensor(rng.standard_normal(n_old), dtype=torch.float64, device="cuda")
        ref = torch.full((n_new,), np.nan, dtype=torch.float64, device="cuda")
        out = torch.full((n_new,), np.nan, dtype=torch.float64, device="cuda")
        tsm.tsm_prolong(lo, ln, vo, ref)
        tsm.tsm_prolong_noalloc(lo, ln, vo, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), n
        assert not torch.isnan(out).any()


def test_noalloc_prolong_refuses_sizes_beyond_its_workspace():
    from paper_2103_17040_amd import tsm
    n = 131073
    lo = np.full(n, 2, np.int32)
    with pytest.raises(tsm.TsmError) as e:
        tsm.tsm_prolong_noalloc(lo, lo, 256, 512, n_old=9 * n, n_new=9 * n)
    assert e.value.status == tsm.TSM_ENOMEM and "131072" in str(e.value)
    # and wrong counts, like tsm_prolong
    with pytest.raises(tsm.TsmError) as e:
        tsm.tsm_prolong_noalloc(lo[:4], lo[:4], 256, 512, n_old=35, n_new=36)
    assert e.value.status == tsm.TSM_EINVAL
