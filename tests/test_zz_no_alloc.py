"""GPU: the allocation-free spectral statistics entry point
(mbf_spectral_stats_noalloc, scratch in a fixed per-device array) against the
allocating one (mbf_spectral_stats) on the same device data, through the C
ABI: two calls in a row, the second smaller, each equal bit for bit, and both
against the oracle's statistics."""
import ctypes

import numpy as np
import pytest

from oracle import spectra as OS
from paper_0809_1547_amd import inputs as I

pytestmark = pytest.mark.gpu


def _dev(F, om):
    import torch
    spec = torch.tensor(np.stack([F.real, F.imag], axis=-1), dtype=torch.float64, device="cuda")
    return spec, torch.tensor(om, dtype=torch.float64, device="cuda")


def test_noalloc_stats_equal_the_allocating_entry_point():
    import torch
    from paper_0809_1547_amd import mbf
    st = torch.cuda.Stream()
    out = torch.zeros(ctypes.sizeof(mbf.mbf_spec_stats), dtype=torch.uint8, device="cuda")
    # the emission spectra of the paper-scale run (256 probes x 874 bins),
    # then a smaller call on the same scratch (7 x 300; the scratch still
    # holds the first call's bins beyond 300)
    for P, K, seed, level in ((256, 874, 21, 0.5), (7, 300, 22, 0.3)):
        F, om = I.synthetic_spectra(P, K, seed=seed, lines=((0.45, 0.03, 1.0), (0.62, 0.01, 0.6)))
        spec, omt = _dev(F, om)
        ref = mbf.mbf_spectral_stats(spec, omt, level, stream=st.cuda_stream)
        with torch.cuda.stream(st):
            out.fill_(0xFF)
            mbf.mbf_spectral_stats_noalloc(spec, omt, out, level, stream=st.cuda_stream)
        st.synchronize()
        got = mbf.spec_stats_from_device(out)
        print(P, K, got["peak_bin"], got["fit_sigma"])
        assert got == ref, (P, K)
        o = OS.spectral_stats(F, om, level)
        for k in ("peak_bin", "fit_lo", "fit_hi", "fit_ok"):
            assert got[k] == o[k], k
        assert got["fit_sigma"] == pytest.approx(o["fit_sigma"], rel=1e-7)
        assert got["std_omega"] == pytest.approx(o["std_omega"], rel=1e-12)


def test_noalloc_stats_reject_sizes_beyond_the_scratch():
    import torch
    from paper_0809_1547_amd import mbf
    spec = torch.zeros((1, 65537, 2), dtype=torch.float64, device="cuda")
    omt = torch.linspace(1.0, 2.0, 65537, dtype=torch.float64, device="cuda")
    out = torch.zeros(ctypes.sizeof(mbf.mbf_spec_stats), dtype=torch.uint8, device="cuda")
    with pytest.raises(mbf.MbfError, match="65536"):
        mbf.mbf_spectral_stats_noalloc(spec, omt, out, 0.5)
    # the largest accepted size works
    F, om = I.synthetic_spectra(2, 65536, seed=23)
    spec, omt = _dev(F, om)
    mbf.mbf_spectral_stats_noalloc(spec, omt, out, 0.5)
    torch.cuda.synchronize()
    assert mbf.spec_stats_from_device(out) == mbf.mbf_spectral_stats(spec, omt, 0.5)
