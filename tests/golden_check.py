"""Comparison of a GPU solution with an oracle solve stored sampled under
tests/golden/ (written by the scripts there, which call only the oracle)."""
import os

import numpy as np
import torch

from paper_2209_06916_amd import inputs


def golden(name):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    with np.load(path) as z:
        return {k: z[k] for k in z.files}


def time_point_tol(n):
    """Per-time-point bar for solutions n steps from t = 0: 1e-12, or 2 n u
    (u = 2^-53) where that is larger.  Two implementations that round each
    application of the same non-expansive step differently drift apart by up
    to about n u after n dependent steps, so past n = 4096 the bar grows with
    n (at n = 16384 it is 3.6e-12)."""
    return np.maximum(1e-12, 2.0 * np.asarray(n, dtype=float) * 2.0 ** -53)


def check_against_golden(info, out, g, c_sample, m, w_seed, row_sample=None):
    """The oracle's full-size solve, stored sampled (see the scripts that
    write the golden files): identical iteration count, residual history,
    per-time-point norms and projections, every C-point's sampled values
    (c_sample: the same sampling of the GPU solution, C-points every m steps)
    and a few time points (sampled by row_sample as the golden file stores
    them), each within time_point_tol."""
    assert info["iterations"] == int(g["iterations"])
    np.testing.assert_allclose(info["res_history"], g["res_history"], rtol=1e-8, atol=1e-14 * g["res_history"][0])
    flat = out.reshape(out.shape[0], -1)
    tol_t = time_point_tol(np.arange(flat.shape[0]))
    norms = torch.linalg.vector_norm(flat, dim=1).cpu().numpy()
    e_norm = np.abs(norms - g["norms"]) / g["norms"] / tol_t
    # <w, e_n> for a random sign vector w is about ||e_n||: 1e-12 of ||u_n||
    # per time point, with a factor 8 for the spread of a random projection
    w = torch.from_numpy(inputs.sign_vector(flat.shape[1], w_seed)).to(out.device)
    proj = (flat @ w).cpu().numpy()
    e_proj = np.abs(proj - g["proj"]) / g["norms"] / (8 * tol_t)
    ref_s = g["c_sample"].reshape(len(g["c_sample"]), -1)
    got_s = c_sample.reshape(len(c_sample), -1)
    e_c = np.linalg.norm(got_s - ref_s, axis=1) / np.linalg.norm(ref_s, axis=1) / tol_t[::m]
    rows = out[torch.from_numpy(g["row_index"]).to(out.device)]
    rows = (row_sample(rows) if row_sample else rows).cpu().numpy()
    ref_r = g["rows"].reshape(len(g["rows"]), -1)
    e_r = (np.linalg.norm(rows.reshape(len(rows), -1) - ref_r, axis=1) / np.linalg.norm(ref_r, axis=1) /
           tol_t[g["row_index"]])
    print("error / bar: norms %.2f, projections %.2f, C-point samples %.2f, time points %.2f"
          % (e_norm.max(), e_proj.max(), e_c.max(), e_r.max()))
    assert e_norm.max() <= 1 and e_proj.max() <= 1 and e_c.max() <= 1 and e_r.max() <= 1
