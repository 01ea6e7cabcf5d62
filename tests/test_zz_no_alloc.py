"""The allocation-free exponential (ep_expm_noalloc) against ep_expm, through the C ABI.

Two calls in a row on the library's static scratch, the second with a smaller matrix (the
array keeps the first call's contents), then an LDS-sized matrix and the size limit."""
import numpy as np
import pytest

from paper_2405_05213_amd import ep as epmod
from tests.gpu_util import pair, say
from workloads import config

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _hessenberg(m, norm1, seed):
    rng = np.random.default_rng(seed)
    H = np.triu(rng.normal(size=(m, m)), -1)
    return H * (norm1 / np.abs(H).sum(axis=0).max())


def test_expm_noalloc_matches_expm():
    ctx, _ = pair(config("c1"), m_max=256)
    stream = torch.cuda.current_stream().cuda_stream
    # 200 and 96 use the device scratch (too large for LDS), 40 runs in LDS
    for m, nrm, seed in [(200, 900.0, 1), (96, 300.0, 2), (40, 50.0, 3)]:
        say(f"[expm_noalloc] m={m} ||H||_1={nrm}")
        H = _hessenberg(m, nrm, seed)
        ref = ctx.expm(H)
        Hd = torch.as_tensor(H, dtype=torch.float64, device=DEV).contiguous()
        Ed = torch.full((m, m), float("nan"), dtype=torch.float64, device=DEV)
        epmod.expm_noalloc(m, Hd, Ed, stream)
        torch.cuda.synchronize()
        E = Ed.cpu().numpy()
        err = np.abs(E - ref).max() / np.abs(ref).max()
        say(f"  max |E - E_ref| / max |E_ref| = {err:.3e}")
        assert np.isfinite(E).all()
        assert err <= 1e-13


def test_expm_noalloc_rejects_sizes_beyond_its_scratch():
    Hd = torch.zeros((257, 257), dtype=torch.float64, device=DEV)
    Ed = torch.zeros_like(Hd)
    for m in (0, 257):
        with pytest.raises(epmod.EPError) as e:
            epmod.expm_noalloc(m, Hd, Ed)
        assert e.value.code == epmod.EP_ERR_ARG
    with pytest.raises(epmod.EPError) as e:
        epmod.expm_noalloc(4, None, Ed)
    assert e.value.code == epmod.EP_ERR_ARG
