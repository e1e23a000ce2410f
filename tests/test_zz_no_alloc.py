"""The allocation-free registration (misslam_gn_register_noalloc) against misslam_gn_register.

Both run the same kernels with the same arithmetic on the same inputs, so parameters, reports and
correspondence histories must agree bit for bit.  Two calls in a row share the one scratch array: the
320x240 frame first, then the smaller 64x48 frame, then the 320x240 frame again over what the smaller one
left behind.
"""
import numpy as np
import pytest
import torch

from gpu_util import Scene

pytestmark = pytest.mark.gpu


def _both(s):
    M = s.M
    x_ref = M.identity_params(s.m)
    rep_ref, ch_ref = M.gn_register(s.pts, s.nodes, x_ref, s.graph, s.depth, s.cam, s.pose, s.params, s.ws,
                                    corr_hist=True)
    x = M.identity_params(s.m)
    rep, ch = M.gn_register_noalloc(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, corr_hist=True)
    torch.cuda.synchronize()
    return (x.cpu().numpy(), M.read_report(rep), ch.cpu().numpy()), \
           (x_ref.cpu().numpy(), M.read_report(rep_ref), ch_ref.cpu().numpy())


def _same(got, ref, name):
    (x, r, ch), (xr, rr, chr_) = got, ref
    print(name, "noalloc vs workspace: params bitwise", np.array_equal(x.view(np.uint32), xr.view(np.uint32)),
          "final e_data", r[-1]["e_data"], rr[-1]["e_data"])
    assert np.array_equal(x.view(np.uint32), xr.view(np.uint32)), name
    assert r.tobytes() == rr.tobytes(), name
    assert np.array_equal(ch, chr_), name
    assert np.all(r["flags"] == 0), name


def test_noalloc_equals_workspace_entry_two_calls(lib):
    big = Scene("c2")
    small = Scene("c1")
    _ = big.graph, small.graph
    _same(*_both(big), "320x240")
    _same(*_both(small), "64x48 after 320x240")
    _same(*_both(big), "320x240 again")
