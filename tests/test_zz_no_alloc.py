"""The no-allocation norm (sv_norm_fp64_noalloc) through the C ABI.

It must give the FP64 norm of sv_norm_fp64 bit for bit, on consecutive calls
whose states differ in size (the fixed partial array keeps the last call's
contents), and refuse out-of-range sizes before touching the device.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1804_04797_amd import qsv  # noqa: E402

pytestmark = pytest.mark.gpu


def _state(n, seed):
    g = torch.Generator().manual_seed(seed)
    re = torch.randn(1 << n, generator=g, dtype=torch.float32)
    im = torch.randn(1 << n, generator=g, dtype=torch.float32)
    return torch.complex(re, im).to("cuda:0")


@pytest.mark.parametrize("sizes", [(26, 20), (22, 16)])
def test_noalloc_norm_matches_norm(sizes):
    dev = torch.device("cuda:0")
    for k, n in enumerate(sizes):
        a = _state(n, 1000 + 7 * k + n)
        want = torch.zeros(1, dtype=torch.float64, device=dev)
        got = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
        qsv.sv_norm_fp64(a, n, want)
        qsv.sv_norm_fp64_noalloc(a, n, got)
        torch.cuda.synchronize()
        w, g = want.item(), got.item()
        assert g == w, (n, g, w)
        # and against the host: FP64 sum of the exact FP64 squares
        h = a.cpu().numpy().astype(np.complex128)
        ref = float(np.sum(h.real * h.real + h.imag * h.imag))
        assert abs(g - ref) <= 1e-12 * ref


def test_noalloc_norm_rejects_out_of_range():
    dev = torch.device("cuda:0")
    a = _state(10, 5)
    out = torch.zeros(1, dtype=torch.float64, device=dev)
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_norm_fp64_noalloc(a, 35, out)
    assert e.value.status == 2
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_norm_fp64_noalloc(None, 10, out)
    assert e.value.status == 1
