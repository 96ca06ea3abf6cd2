"""Writes ``c5_oracle_sample.npz``: the FP64 oracle's first roots, normals and
flags at a fixed set of pixels of the 16384-primitive 3840x2160 frame
(scenegen.config5, seed 7777).

Tracing the full 32,767-node tree in FP64 costs about a third of a
core-second per ray, so the GPU test of that frame reads these stored values instead of
recomputing thousands of rays.  Everything here comes from the scene
generator and the oracle; the pixels are chosen without any GPU output:

* 512 seeded uniform pixels of the frame;
* a lattice of every 16th pixel in both directions (seeded phase);
* the hit regions found on that lattice, filled at a stride of 2 pixels:
  starting from the lattice hits, the stride-2 neighbours of every hit are
  traced in turn until 2,400 hits are reached or no region grows (the frame
  is about 0.2% hit in small scattered regions, so a uniform sample would
  hold about one hit in 400 rays).

Run: ``python tests/golden/make_c5_oracle.py`` (about 30 minutes on 8 cores).
The file records a digest of the scene arrays and camera; the test refuses a
stale file.
"""
from __future__ import annotations

import hashlib
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402
import scenegen as sg  # noqa: E402

OUT = Path(__file__).resolve().parent / "c5_oracle_sample.npz"


def scene_digest(sc) -> str:
    h = hashlib.sha256()
    for a in (sc.kind, sc.left, sc.right, sc.params):
        h.update(np.ascontiguousarray(a).tobytes())
    c = sc.camera
    h.update(np.array([*c.eye, *c.target, *c.up, c.vfov_deg, c.width, c.height], dtype=np.float64).tobytes())
    h.update(np.int64(sc.root).tobytes())
    return h.hexdigest()


def trace(osc, cam, px, py, label):
    t0 = time.time()
    t, nrm, flag, _ = osc.trace(cam, px.astype(np.float64) + 0.5, py.astype(np.float64) + 0.5)
    print(f"{label}: {px.shape[0]} rays, {int((flag & 1).sum())} hits, {time.time() - t0:.0f} s", flush=True)
    return t, nrm, flag


def main():
    sc = sg.config5()
    cam = sc.camera
    W, H = cam.width, cam.height
    osc = oracle.OracleScene(sc)
    rng = np.random.default_rng(20240417)

    rand = rng.choice(W * H, size=512, replace=False)
    oy, ox = rng.integers(0, 16, 2)
    gy, gx = np.mgrid[oy:H:16, ox:W:16]
    lat = np.setdiff1d((gy * W + gx).ravel(), rand)

    chunks = []
    t, n, f = trace(osc, cam, rand % W, rand // W, "uniform")
    chunks.append((rand, t, n, f))
    t, n, f = trace(osc, cam, lat % W, lat // W, "lattice")
    chunks.append((lat, t, n, f))

    seen = set(rand.tolist()) | set(lat.tolist())
    hits = [c[0][(c[3] & 1) != 0] for c in chunks]
    n_hits = sum(h.shape[0] for h in hits)
    front = np.concatenate(hits)
    rnd = 0
    while n_hits < 2400 and front.shape[0] > 0:
        nb = []
        for dy, dx in ((-2, 0), (2, 0), (0, -2), (0, 2)):
            r, c = front // W + dy, front % W + dx
            ok = (r >= 0) & (r < H) & (c >= 0) & (c < W)
            nb.append((r * W + c)[ok])
        nb = np.unique(np.concatenate(nb))
        nb = np.array([q for q in nb.tolist() if q not in seen], dtype=np.int64)
        if nb.shape[0] == 0:
            break
        seen.update(nb.tolist())
        rnd += 1
        t, n, f = trace(osc, cam, nb % W, nb // W, f"fill round {rnd}")
        chunks.append((nb, t, n, f))
        front = nb[(f & 1) != 0]
        n_hits += front.shape[0]

    idx = np.concatenate([c[0] for c in chunks])
    order = np.argsort(idx)
    np.savez_compressed(
        OUT,
        digest=np.array(scene_digest(sc)),
        px=(idx % W).astype(np.int32)[order], py=(idx // W).astype(np.int32)[order],
        t=np.concatenate([c[1] for c in chunks])[order],
        normal=np.concatenate([c[2] for c in chunks])[order],
        flag=np.concatenate([c[3] for c in chunks]).astype(np.int32)[order],
        extent=np.float64(osc.extent),
    )
    fl = np.concatenate([c[3] for c in chunks])
    print(f"wrote {OUT}: {idx.shape[0]} pixels, {int((fl & 1).sum())} hits, "
          f"{int((fl & 2).sum() // 2)} undecided")


if __name__ == "__main__":
    main()
