"""ap_nblist_build_noalloc (no context; scratch in a static device array) against ap_nblist_build and the
oracle: the same neighbour sets, bit for bit, on calls in a row whose later inputs are smaller, with an
overflow in between (the scratch keeps the last call's contents, so each call must clear what it needs)."""
import numpy as np
import pytest

import synth
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _sets(cnt, idx):
    cnt, idx = cnt.cpu().numpy(), idx.cpu().numpy()
    return [np.sort(idx[:cnt[i], i]) for i in range(len(cnt))]


def _check(oracle, pos, box, r, m):
    import torch
    from paper_2512_07693_amd import ap
    n = len(pos)
    print("noalloc list n=%d r=%.1f max_nbr=%d" % (n, r, m), flush=True)
    P = to_dev(pos)
    ctx = ap.Context(n, max_nbr=m)
    c_ref, i_ref = ctx.nblist_build(P, box, r, m)
    cnt = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    idx = torch.full((m, n), -1, dtype=torch.int32, device="cuda")
    ap.nblist_build_noalloc(P, box, r, cnt, idx)
    torch.cuda.synchronize()
    assert np.array_equal(cnt.cpu().numpy(), c_ref.cpu().numpy())
    got, ref = _sets(cnt, idx), _sets(c_ref, i_ref)
    want = oracle.nblist(pos, box, r, cap=m)
    for i in range(n):
        assert np.array_equal(got[i], ref[i]) and np.array_equal(got[i], want[i]), i
    ctx.close()


def test_noalloc_list_matches_context_list(oracle):
    import torch
    from paper_2512_07693_amd import ap
    s = synth.build_system(1)  # 1,024 bcc atoms with a hot spot
    _check(oracle, s["pos"], s["box"], 7.0, 160)
    # an overflow: reported, and the next call starts clean
    P = to_dev(s["pos"])
    cnt = torch.zeros(len(s["pos"]), dtype=torch.int32, device="cuda")
    idx = torch.zeros((20, len(s["pos"])), dtype=torch.int32, device="cuda")
    with pytest.raises(ap.APError) as e:
        ap.nblist_build_noalloc(P, s["box"], 7.0, cnt, idx)
    assert e.value.code == -3
    # a smaller input next: 250 atoms, and lists longer than the 256 slots the staged build takes
    rng = np.random.default_rng(5)
    ref, box = synth.bcc(3.16, 5)
    small = synth.gaussian_displace(ref, 0.1, rng)
    _check(oracle, small, box, 6.0, 96)
    _check(oracle, small, box, 7.5, 300)


def test_noalloc_list_rejects_inputs_beyond_the_scratch():
    import torch
    from paper_2512_07693_amd import ap
    n = (1 << 17) + 1
    P = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    idx = torch.zeros((8, n), dtype=torch.int32, device="cuda")
    with pytest.raises(ap.APError) as e:
        ap.nblist_build_noalloc(P, [400.0, 400.0, 400.0], 6.0, cnt, idx)
    assert e.value.code == -1 and "131072" in str(e.value)
