"""Helpers of the GPU parity tests: run the library on a scene and compare
with the FP64 oracle under the parity rules (hit/miss exact, depth within
1e-4 of the scene extent, normals within 1e-3 rad; rays within 1e-4 of a
silhouette and rays at sharp creases are exempt where the rules say so)."""
from __future__ import annotations

import numpy as np

import oracle

DEPTH_REL_TOL = 1e-4      # of the scene extent
NORMAL_TOL = 1e-3         # radians
SIL_OFFSET = 1e-4         # scene units


def gpu_render(sc, tuning=None):
    import torch
    from paper_2304_09673_amd import st
    s = st.Scene(sc)
    s.build_abuffer(sc.camera, tuning)
    d, n, stats = s.trace()
    torch.cuda.synchronize()
    return s, d.cpu().numpy(), n.cpu().numpy(), stats


def compare(sc, depth, normal, px, py, osc=None):
    """Parity of GPU outputs at integer pixels (px, py) against the oracle.
    Returns a dict of counts; 'fail' must be 0."""
    osc = osc or oracle.OracleScene(sc)
    cam = sc.camera
    fx, fy = px.astype(np.float64) + 0.5, py.astype(np.float64) + 0.5
    t, nrm, flag, _ = osc.trace(cam, fx, fy)
    hit_o = (flag & 1) != 0
    undecided = (flag & 2) != 0
    crease = (flag & 4) != 0
    tg = depth[py, px].astype(np.float64)
    ng = normal[py, px].astype(np.float64)
    hit_g = np.isfinite(tg)
    tol = DEPTH_REL_TOL * osc.extent
    both = hit_o & hit_g
    dz = np.where(both, np.abs(tg - np.where(hit_o, t, 0)), 0.0)
    cosang = np.clip(np.sum(ng * nrm, axis=1), -1.0, 1.0)
    ang = np.where(both, np.arccos(cosang), 0.0)
    mask_bad = hit_o != hit_g
    depth_bad = both & (dz > tol)
    normal_bad = both & ~crease & (ang > NORMAL_TOL)
    suspect = (mask_bad | depth_bad | normal_bad) & ~undecided
    exempt = np.zeros_like(suspect)
    if suspect.any():
        idx = np.nonzero(suspect)[0]
        exempt[idx] = oracle.silhouette_flags(osc, cam, fx[idx], fy[idx], np.where(hit_o, t, np.inf)[idx],
                                              hit_o[idx], tol, SIL_OFFSET)
    fail = suspect & ~exempt
    return {
        "rays": int(px.shape[0]), "hits_oracle": int(hit_o.sum()), "hits_gpu": int(hit_g.sum()),
        "mask_mismatch": int(mask_bad.sum()), "depth_bad": int(depth_bad.sum()), "normal_bad": int(normal_bad.sum()),
        "exempt": int((suspect & exempt).sum()), "undecided": int(undecided.sum()), "crease": int(crease.sum()),
        "fail": int(fail.sum()), "fail_idx": np.nonzero(fail)[0][:20].tolist(),
        "max_depth_err_rel": float(dz[both & ~suspect].max() / osc.extent) if (both & ~suspect).any() else 0.0,
        "max_normal_err": float(ang[both & ~crease & ~suspect].max()) if (both & ~crease & ~suspect).any() else 0.0,
        "extent": osc.extent,
    }


def all_pixels(cam):
    jj, ii = np.mgrid[0:cam.height, 0:cam.width]
    return ii.ravel(), jj.ravel()


def sample_pixels(cam, n, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, cam.width, n), rng.integers(0, cam.height, n)
