"""nep_spin_eval_noalloc (every device buffer in the library's static
scratch array, no device allocation) against nep_spin_eval, through the C
ABI: two calls in a row, the second on a smaller system, then a system too
large for the scratch array."""
import ctypes as ct

import numpy as np
import pytest

from paper_2606_14073_amd import workload as W

pytestmark = pytest.mark.gpu


def _eval(nepspin, model, s, prec, noalloc, device=False):
    """E, E_i, F, H through the C entry point, host or device buffers"""
    v, keep = nepspin.system_view(s.types, s.pos, s.spin, s.box, s.pbc, 1.0, (0.1, -0.2, 0.6))
    fn = nepspin.load().nep_spin_eval_noalloc if noalloc else nepspin.load().nep_spin_eval
    prec_code = nepspin.PRECISION[prec]
    if not device:
        E, Ei, F, H = np.zeros(1), np.zeros(s.n), np.zeros((s.n, 3)), np.zeros((s.n, 3))
        p = [a.ctypes.data_as(ct.c_void_p) for a in (E, Ei, F, H)]
        rc = fn(model.h, ct.byref(v), prec_code, *p, None)
        return rc, (E[0], Ei, F, H)
    import torch
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    Ei = torch.zeros(s.n, dtype=torch.float64, device="cuda")
    F = torch.zeros(s.n, 3, dtype=torch.float64, device="cuda")
    H = torch.zeros(s.n, 3, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    ex = nepspin.Exec(1, ct.c_void_p(stream) if stream else None)
    rc = fn(model.h, ct.byref(v), prec_code, *[ct.c_void_p(t.data_ptr()) for t in (E, Ei, F, H)], ct.byref(ex))
    torch.cuda.synchronize()
    return rc, (E.item(), Ei.cpu().numpy(), F.cpu().numpy(), H.cpu().numpy())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_eval_two_calls(prec):
    from paper_2606_14073_amd import nepspin
    model = nepspin.Model(W.random_params(), short_range=W.SHORT_RANGE_FEGE)
    for cells, device in (((8, 8, 8), False), ((4, 4, 4), True)):
        s = W.fege_lattice(*cells, noise=0.05)
        print(f"{prec}: {s.n} atoms, device buffers {device}", flush=True)
        rc0, ref = _eval(nepspin, model, s, prec, False)
        assert rc0 == 0
        rc1, got = _eval(nepspin, model, s, prec, True, device=device)
        assert rc1 == 0, nepspin.load().sl_last_error()
        assert got[0] == ref[0]
        for a, b in zip(got[1:], ref[1:]):
            assert np.array_equal(a, b)
    model.close()


def test_noalloc_rejects_oversize():
    from paper_2606_14073_amd import nepspin
    model = nepspin.Model(W.random_params())
    s = W.fege_lattice(12, 12, 12)
    rc, _ = _eval(nepspin, model, s, "fp64", True)
    assert rc == nepspin.SL_E_OOM
    assert b"scratch" in nepspin.load().sl_last_error()
    # the scratch array is still usable afterwards
    s = W.config_small()
    rc0, ref = _eval(nepspin, model, s, "fp64", False)
    rc1, got = _eval(nepspin, model, s, "fp64", True)
    assert rc0 == 0 and rc1 == 0
    assert np.array_equal(got[2], ref[2]) and got[0] == ref[0]
    model.close()
