"""Noise schedule of the forward diffusion process (Section IV-B).

The forward kernel is N(sqrt(alpha_i) tau_{i-1}, (1 - alpha_i) I) and
alpha-bar_i is the product of alpha_1..alpha_i (the line after Eq. denoising).
The betas are linear from beta_min to beta_max, both ends included, over
i = 1..N (our reading; the paper does not print its schedule).  alpha-bar_0 = 1.

Pinned by exact rational products (tests/test_oracle_schedule.py).
"""
import numpy as np


def betas(n_steps, beta_min, beta_max):
    """beta_i for i = 1..N as an array of length N (index 0 is step 1)."""
    if n_steps == 1:
        return np.array([float(beta_min)])
    i = np.arange(n_steps, dtype=np.float64)
    return float(beta_min) + (float(beta_max) - float(beta_min)) * i / (n_steps - 1)


def alpha_bar(n_steps, beta_min, beta_max):
    """alpha-bar_i for i = 0..N (length N + 1, alpha-bar_0 = 1)."""
    a = 1.0 - betas(n_steps, beta_min, beta_max)
    out = np.empty(n_steps + 1)
    out[0] = 1.0
    prod = 1.0
    for i in range(1, n_steps + 1):
        prod = prod * a[i - 1]
        out[i] = prod
    return out


def step_scalars(n_steps, beta_min, beta_max):
    """Per-step scalars of Algorithm 1, indexed by i = 0..N (row 0 unused).

    mean_scale_i = 1 / sqrt(alpha-bar_i): centre of the sample distribution (Eq. mc)
    sigma_i      = sqrt(1 / alpha-bar_i - 1): its standard deviation (Eq. mc)
    out_scale_i  = sqrt(alpha-bar_{i-1}): factor of the one-step update (Eq. mbd-denoising)
    """
    ab = alpha_bar(n_steps, beta_min, beta_max)
    ms = np.zeros(n_steps + 1)
    sg = np.zeros(n_steps + 1)
    os_ = np.zeros(n_steps + 1)
    for i in range(1, n_steps + 1):
        ms[i] = 1.0 / np.sqrt(ab[i])
        sg[i] = np.sqrt(1.0 / ab[i] - 1.0)
        os_[i] = np.sqrt(ab[i - 1])
    return ms, sg, os_
