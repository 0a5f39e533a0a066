"""Denoising of Section 3.2 on the CPU: the oracle's patch coding and overlap averaging pinned to
closed forms (a complete orthonormal basis reproduces the image exactly; a constant image is a
single DC atom per patch), the overcomplete DCT start of Section 3.2.1, and the PSNR figure."""
import numpy as np

import oracle
from paper_1403_4781_amd import evaluate, synth


def _orthonormal_dct2(p):
    n = np.arange(p)
    C = np.cos(np.pi * np.outer(n + 0.5, n) / p)        # DCT-II basis vectors as columns
    C /= np.linalg.norm(C, axis=0)
    return np.kron(C, C).T                              # (p*p, p*p), orthonormal rows


def test_odct_structure():
    D = synth.odct(8, 16, 16)
    assert D.shape == (256, 64)
    np.testing.assert_allclose(np.linalg.norm(D, axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(D[0], 1.0 / 8.0, atol=1e-14)          # the constant (DC) atom
    # separable: every atom is an outer product of two one-dimensional atoms
    for k in (1, 17, 100, 255):
        A = D[k].reshape(8, 8)
        assert np.linalg.matrix_rank(A, tol=1e-12) == 1
    # every atom but the DC one has zero mean
    assert np.abs(D[1:].sum(axis=1)).max() < 1e-12
    assert synth.odct(8, 16, 8).shape == (128, 64)


def test_denoise_reproduces_image_with_complete_basis():
    rng = np.random.default_rng(601)
    img = rng.uniform(0, 255, (20, 17))
    D = _orthonormal_dct2(4)
    out, codes = oracle.denoise(img, D, 4, 1e-9, 16)
    np.testing.assert_allclose(out, img, atol=1e-8)
    assert codes.idx.shape[0] == 17 * 14


def test_denoise_constant_image_is_one_atom_per_patch():
    img = np.full((30, 26), 100.0)
    D = synth.odct(8, 16, 16)
    out, codes = oracle.denoise(img, D, 8, 1e-6, 8)
    np.testing.assert_allclose(out, 100.0, atol=1e-10)
    assert (codes.nnz == 1).all() and (codes.idx[:, 0] == 0).all()


def test_psnr_closed_form():
    clean = np.random.default_rng(603).uniform(0, 255, (16, 16))
    assert abs(evaluate.psnr(clean, clean + 5.0) - 20 * np.log10(255 / 5.0)) < 1e-12


def test_denoise_reduces_noise_on_a_synthetic_image():
    rng = np.random.default_rng(604)
    clean = synth.synthetic_image(rng, 40, 40)
    noisy = clean + 20.0 * rng.standard_normal(clean.shape)
    out, _ = oracle.denoise(noisy, synth.odct(8, 16, 16), 8, 8.5 * 20.0, 16)
    assert evaluate.psnr(clean, out) > evaluate.psnr(clean, noisy) + 3.0
