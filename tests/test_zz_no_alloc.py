"""The duplicate scan in the library's fixed per-GPU workspace
(hp_find_duplicates_device_static, for callers that cannot allocate) against
the scan in library-allocated workspace (hp_find_duplicates_device): same
pair count and pairs, on two calls in a row, the second on a smaller input
(the workspace keeps the first call's contents)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def planted(P, n, seed):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((P, n)) + 1j * rng.standard_normal((P, n))) * 3
    st = np.zeros(P, np.int32)
    st[::9] = 2
    for k in range(0, P // 2, 89):
        x[k + P // 2] = x[k] * (1 + (3e-7 if k % 2 else 5e-6))
    return x, st


def test_static_scan_matches_allocating_scan():
    import torch
    import paper_1804_03807_amd as hp
    ctx = hp.Context(0)
    try:
        for P, n, seed in ((60000, 7, 1), (5000, 4, 2)):
            x, st = planted(P, n, seed)
            e_d = torch.from_numpy(np.ascontiguousarray(x)).cuda()
            s_d = torch.from_numpy(st).cuda()
            ref_pairs, ref_found = ctx.find_duplicates_device(e_d, s_d, 1e-6, max_pairs=4096)
            pairs = torch.full((4096, 2), -1, dtype=torch.int64, device="cuda")
            found = ctx.find_duplicates_device_static(e_d, s_d, pairs, 1e-6)
            got = {tuple(int(v) for v in p) for p in pairs[:found].cpu().numpy()}
            ref = {tuple(int(v) for v in p) for p in ref_pairs.cpu().numpy()}
            assert found == ref_found and got == ref and len(ref) >= 5
            assert (pairs[found:] == -1).all()
    finally:
        ctx.close()
