"""Checkpoint / resume of a PDFB state (Alg. 1 carries X, P, W and v from one
reweighting pass to the next; with the weights and thresholds that tuple is
the whole state of the iteration).

    save(path, plan, **tensors)   device or host tensors -> one .npz file, with
                                  the plan's configuration and sizes
    load(path, plan, device)      -> dict of contiguous tensors on `device`,
                                  after checking that the file was written for a
                                  plan of the same configuration

Arrays are stored in their own dtype (float32 duals and images, float64
weights and thresholds), so a resumed run continues bit for bit.  Only plain
arrays are written (no pickled objects); the file is read with
allow_pickle=False.
"""
import json

import numpy as np

from .binding import FhsError


def _config(plan):
    c = plan.cfg
    return {"ny": c.ny, "nx": c.nx, "nchan": c.nchan, "qy": c.qy, "qx": c.qx, "n_sub": c.n_sub,
            "overlap_y": c.overlap_y, "overlap_x": c.overlap_x, "levels": c.levels}


def save(path, plan, **tensors):
    arrays = {}
    for name, t in tensors.items():
        if name.startswith("_"):
            raise FhsError(f"checkpoint: array name {name!r} is reserved")
        a = t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)
        arrays[name] = np.ascontiguousarray(a)
    meta = {"config": _config(plan), "sizes": dict(plan.sizes), "arrays": sorted(arrays)}
    arrays["_meta"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    with open(path, "wb") as fh:
        np.savez(fh, **arrays)


def load(path, plan, device="cuda"):
    import torch
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(bytes(z["_meta"]).decode())
        if meta["config"] != _config(plan):
            raise FhsError(f"checkpoint: written for plan {meta['config']}, not {_config(plan)}")
        return {name: torch.from_numpy(np.array(z[name])).to(device) for name in meta["arrays"]}
