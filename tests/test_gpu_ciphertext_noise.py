"""The paper's check that an encrypted FITS payload looks like noise: the
byte histogram of the FITS-shaped plaintext is far from uniform (big-endian
float32 sky levels near 1000 ADU), and that of its AES-256-GCM ciphertext,
made by the HIP path, is not distinguishable from uniform by a chi-square
test.  The ciphertext itself is pinned to the oracle elsewhere; here only
its statistics are checked (a fixed seeded input, so the statistic is a
fixed number, ~255 +- 23 for uniform bytes)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2602_23067_amd import gcm, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

# chi-square with 255 degrees of freedom: mean 255, standard deviation 22.6;
# 400 is more than six standard deviations above the mean
UNIFORM_CHI2_MAX = 400.0


def _chi2(counts):
    counts = counts.astype(np.float64)
    expected = counts.sum() / 256.0
    return float(((counts - expected) ** 2 / expected).sum())


def test_fits_ciphertext_bytes_look_uniform():
    msg = workloads.config2(ny=2048, nx=2048, n_sources=500)  # 16 MiB of FITS-shaped pixels
    print(f"noise check: {msg.data.size} bytes", flush=True)
    ctx = gcm.Context(device=0, key_slots=4)
    try:
        pt = torch.from_numpy(msg.data).cuda()
        aad = torch.from_numpy(msg.aad).cuda()
        ct = torch.empty_like(pt)
        ctx.encrypt(msg.key, msg.iv, aad, pt, ct)
        torch.cuda.synchronize()
        pt_chi2 = _chi2(torch.bincount(pt.long(), minlength=256).cpu().numpy())
        ct_chi2 = _chi2(torch.bincount(ct.long(), minlength=256).cpu().numpy())
    finally:
        torch.cuda.synchronize()
        ctx.close()
    assert pt_chi2 > 1e6, f"the FITS-shaped plaintext should be far from uniform (chi2 {pt_chi2:.0f})"
    assert ct_chi2 < UNIFORM_CHI2_MAX, f"ciphertext byte histogram chi2 {ct_chi2:.1f} >= {UNIFORM_CHI2_MAX}"
