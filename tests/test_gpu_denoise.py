"""GPU denoising (Section 3.2.2) against the FP64 oracle on the same noisy image and dictionary.
Patches whose FP32 residual lands on the other side of eps than the FP64 one take one atom more
or less; their estimates move a few grey levels on their pixels, so the images are compared by
the fraction of pixels that agree closely and by the PSNR of one against the other."""
import numpy as np
import pytest
import torch

import oracle
from paper_1403_4781_amd import evaluate, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h(dev):
    import paper_1403_4781_amd as smdl
    return smdl.Handle(0)


@pytest.mark.parametrize("H,W,sigma", [(64, 56, 20.0), (41, 77, 10.0)])
def test_denoise_against_oracle(h, dev, H, W, sigma):
    print(f"case denoise {H}x{W} sigma={sigma}", flush=True)
    rng = np.random.default_rng(700 + H)
    clean = synth.synthetic_image(rng, H, W)
    noisy = (clean + sigma * rng.standard_normal(clean.shape)).astype(np.float32)
    D = synth.odct(8, 16, 16).astype(np.float32)
    eps = 8.5 * sigma
    ref, codes = oracle.denoise(noisy, D, 8, eps, 16)
    out = h.denoise(torch.from_numpy(noisy).to(dev), torch.from_numpy(D).to(dev), 8, eps, 16).cpu().numpy()
    close = np.abs(out - ref) <= 0.05
    agree = evaluate.psnr(ref, out)
    print(f"  pixels within 0.05: {close.mean():.4f}; PSNR gpu vs oracle {agree:.1f} dB; "
          f"denoised {evaluate.psnr(clean, out):.2f} dB (oracle {evaluate.psnr(clean, ref):.2f}, noisy "
          f"{evaluate.psnr(clean, noisy):.2f})", flush=True)
    assert close.mean() >= 0.98
    assert agree >= 50.0
    assert abs(evaluate.psnr(clean, out) - evaluate.psnr(clean, ref)) <= 0.05


def test_denoise_argument_errors(h, dev):
    import paper_1403_4781_amd as smdl
    img = torch.zeros((20, 20), device=dev)
    D = torch.from_numpy(synth.odct(8, 16, 16).astype(np.float32)).to(dev)
    with pytest.raises(smdl.SmdlError):
        h.denoise(img, D, 8, 0.0, 8)                       # eps must be positive
    with pytest.raises(smdl.SmdlError):
        h.denoise(torch.zeros((6, 20), device=dev), D, 8, 1.0, 8)   # smaller than a patch
    with pytest.raises(smdl.SmdlError):
        h.denoise(img, D, 8, 1.0, 65)                      # s_max beyond min(m, K)
