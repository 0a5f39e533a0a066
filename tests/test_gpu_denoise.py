"""GPU denoising (Section 3.2.2) against the FP64 oracle on the same noisy image and dictionary.

The patch codes are compared element by element (the parity bar of the OMP tests, with the
error-constrained tie rule: patches whose FP64 residual passes within 1e-5 ||y|| of eps at some
step may stop one atom earlier or later in FP32).  Every pixel that no such patch covers must
then agree with the oracle's image to 1e-7 of the largest patch norm: the estimates carry FP32
rounding of the coefficients and of the averaging only (a few 2^-24 of the pixel values).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1403_4781_amd import evaluate, synth
from tests.parity import compare, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h(dev):
    import paper_1403_4781_amd as smdl
    return smdl.Handle(0)


def _patches(img, p):
    """Every p x p patch (stride 1), row-major patch order, each flattened row-major."""
    v = np.lib.stride_tricks.sliding_window_view(img, (p, p))
    return np.ascontiguousarray(v.reshape(-1, p * p))


@pytest.mark.parametrize("H,W,sigma", [(64, 56, 20.0), (41, 77, 10.0)])
def test_denoise_against_oracle(h, dev, H, W, sigma):
    print(f"case denoise {H}x{W} sigma={sigma}", flush=True)
    rng = np.random.default_rng(700 + H)
    clean = synth.synthetic_image(rng, H, W)
    noisy = (clean + sigma * rng.standard_normal(clean.shape)).astype(np.float32)
    D = synth.odct(8, 16, 16).astype(np.float32)
    eps = 8.5 * sigma
    ref, _ = oracle.denoise(noisy, D, 8, eps, 16)
    Dt = torch.from_numpy(D).to(dev)
    out = h.denoise(torch.from_numpy(noisy).to(dev), Dt, 8, eps, 16).cpu().numpy()
    # the patch codes, element by element
    P = _patches(noisy, 8)
    ora = oracle.omp(D, P, 16, eps=eps, trace=True)
    X = h.omp_code(Dt, torch.from_numpy(P).to(dev), 16, eps=eps)
    compare(to_np(X), ora, D, P, eps=eps, label=f"denoise patches {H}x{W}")
    # pixels covered only by patches away from the eps boundary
    ties = oracle.tie_mask(ora, eps=eps)
    PW = W - 7
    cover = np.zeros((H, W), bool)
    for n in np.flatnonzero(ties):
        cover[n // PW:n // PW + 8, n % PW:n % PW + 8] = True
    tol = 1e-7 * float(np.linalg.norm(P.astype(np.float64), axis=1).max())
    err = np.abs(out.astype(np.float64) - ref)
    print(f"  tie patches {int(ties.sum())} of {len(P)}, pixels they cover {int(cover.sum())} of {H * W}; "
          f"max error elsewhere {err[~cover].max():.2e} (bound {tol:.2e}); denoised "
          f"{evaluate.psnr(clean, out):.2f} dB (oracle {evaluate.psnr(clean, ref):.2f}, noisy "
          f"{evaluate.psnr(clean, noisy):.2f})", flush=True)
    assert (err[~cover] <= tol).all()
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
