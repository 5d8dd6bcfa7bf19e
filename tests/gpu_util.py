"""Shared helpers of the GPU tests: device transfer and the parity bar.

Parity bar (per masked node): |gamma_gpu - gamma_oracle| <= 1e-5 + 1e-5 * gamma_oracle;
identical masks; identical pass decisions (gamma <= 1) except for nodes whose oracle
gamma lies within 1e-5 of 1, which are counted separately.
"""
import numpy as np

ATOL = 1e-5
RTOL = 1e-5
BAND = 1e-5


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def assert_parity(g_gpu: np.ndarray, g_ref: np.ndarray, label: str = ""):
    """Compare a GPU gamma map (float32) with oracle gammas (float64) of the same nodes."""
    g_gpu = np.asarray(g_gpu, dtype=np.float64).ravel()
    g_ref = np.asarray(g_ref, dtype=np.float64).ravel()
    assert g_gpu.shape == g_ref.shape
    m_ref = g_ref >= 0
    m_gpu = g_gpu >= 0
    assert np.array_equal(m_ref, m_gpu), f"{label}: masks differ ({m_ref.sum()} vs {m_gpu.sum()})"
    err = np.abs(g_gpu[m_ref] - g_ref[m_ref])
    bound = ATOL + RTOL * g_ref[m_ref]
    bad = err > bound
    if bad.any():
        k = np.argmax(err - bound)
        raise AssertionError(f"{label}: {bad.sum()} nodes beyond tolerance; worst |d|={err[k]:.3e} "
                             f"at gamma={g_ref[m_ref][k]:.6f}")
    outside = m_ref & (np.abs(g_ref - 1.0) > BAND)
    pass_ref = g_ref[outside] <= 1.0
    pass_gpu = g_gpu[outside] <= 1.0
    assert np.array_equal(pass_ref, pass_gpu), f"{label}: pass decisions differ outside the band"
    return float(err.max()) if err.size else 0.0
