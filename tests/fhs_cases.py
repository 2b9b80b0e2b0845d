"""Test helpers: seeded problems in both the library's packed layouts and the
oracle's per-facet structures, and the error measures used by the parity
tests.  (Test infrastructure; imports the oracle and the binding.)"""
import sys

import numpy as np

import synth
from oracle import geometry, heuristics, sara, step


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    d = np.linalg.norm(a - b)
    return d / nb if nb > 0 else d


def max_rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m = np.max(np.abs(b)) if b.size else 0.0
    d = np.max(np.abs(a - b)) if b.size else 0.0
    return d / m if m > 0 else d


class Problem:
    """One seeded problem: cube, duals, weights, thresholds (float32 / float64
    arrays exactly as handed to both sides)."""

    def __init__(self, ny, nx, L, qy=1, qx=1, C=1, oy=0, ox=0, levels=4, seed=0, blobs=50,
                 warm=False, variant="plain", zero=False, sigma_scale=1e-3):
        self.ny, self.nx, self.L, self.C = ny, nx, L, C
        self.Lc = L // C
        self.levels = levels
        self.geom = geometry.Geometry(ny, nx, qy, qx, oy, ox, levels)
        self.cfg = (ny, nx, L, qy, qx, C, oy, ox, levels)
        base = synth.BASE_SEED + 1000 * seed
        if zero:
            X = np.zeros((ny, nx, L), dtype=np.float32)
        else:
            X = synth.blob_cube(ny, nx, L, blobs, base)
            if variant == "signed":
                Xb = synth.blob_cube(ny, nx, L, blobs, base + 1)
                X = (2.0 * X.astype(np.float64) - Xb).astype(np.float32)
        self.X = X
        self.I = sara.n_coefficients(ny, nx, levels)
        Q = self.geom.Q
        sb = sigma_scale * float(np.max(np.abs(X))) if not zero else 1e-3
        self.mu = np.array([heuristics.mu_sparsity(sb, self.Lc)] * C)
        self.mu_bar = np.array([[heuristics.mu_low_rank(sb, f.n_rows, self.Lc) for f in self.geom.facets]
                                for _ in range(C)])
        self.theta = [synth.uniform_weights(self.I, base + 10 + c) for c in range(C)]
        self.theta_bar = [[synth.sorted_weights(self.Lc, base + 100 + c * Q + q) for q in range(Q)]
                          for c in range(C)]
        tscale = float(np.median(self.mu_bar)) if not zero else 1.0
        self.P = []
        for c in range(C):
            row = []
            for q, f in enumerate(self.geom.facets):
                shp = f.nuc_shape + (self.Lc,)
                row.append(synth.gaussian(shp, base + 200 + c * Q + q, 0.1 * tscale / np.sqrt(f.n_rows))
                           if warm else np.zeros(shp, dtype=np.float32))
            self.P.append(row)
        self.W = [synth.gaussian((self.I, self.Lc), base + 300 + c, 0.5 * self.mu[0]) if warm
                  else np.zeros((self.I, self.Lc), dtype=np.float32) for c in range(C)]

    # ---------------------------------------------------------------- packing
    def P_flat(self):
        return np.concatenate([p.reshape(-1) for row in self.P for p in row]).astype(np.float32)

    def P_unflat(self, flat):
        out, off = [], 0
        for c in range(self.C):
            row = []
            for f in self.geom.facets:
                n = f.n_rows * self.Lc
                row.append(flat[off:off + n].reshape(f.nuc_shape + (self.Lc,)))
                off += n
            out.append(row)
        return out

    def W_flat(self):
        return np.concatenate(self.W, axis=1).astype(np.float32).reshape(-1)

    def W_unflat(self, flat):
        Wf = flat.reshape(self.I, self.L)
        return [Wf[:, c * self.Lc:(c + 1) * self.Lc] for c in range(self.C)]

    def theta_flat(self):
        return np.concatenate(self.theta).astype(np.float32)

    def theta_bar_flat(self):
        return np.concatenate([t for row in self.theta_bar for t in row]).astype(np.float64)

    def mu_bar_flat(self):
        return np.asarray(self.mu_bar, dtype=np.float64).reshape(-1)

    # ---------------------------------------------------------------- oracle
    def oracle_step(self, zeta=1.0, kappa=1.0):
        return step.facet_prox_step(self.X, self.P, self.W, self.theta, self.theta_bar, self.mu, self.mu_bar,
                                    zeta, kappa, self.geom, C=self.C)

    def oracle_nuclear(self, zeta=1.0):
        return step.nuclear_dual_update(self.X, self.P, self.theta_bar, self.mu_bar, zeta, self.geom, C=self.C)

    def oracle_l21(self, kappa=1.0):
        return step.l21_dual_update(self.X, self.W, self.theta, self.mu, kappa, self.levels, C=self.C)

    def oracle_analysis(self):
        """Psi^dagger X in the library's [I][L] position layout."""
        outs = []
        for ch in step.subcube_channels(self.L, self.C):
            outs.append(sara.flatten(sara.analysis(self.X.astype(np.float64)[..., ch], self.levels)))
        return np.concatenate(outs, axis=1)


# ---------------------------------------------------------------- full-size problems on the device
def fill_warm_duals(plan, p_dev, w_dev, mu, mu_bar, chunk_rows=1 << 20):
    """Warm duals of a full-size problem written straight into the device
    arrays with the counter-based generator of `synth` (the sampled-block
    oracle evaluates the same values on the host)."""
    import torch
    s = plan.sizes
    C, L, Lc = plan.C, plan.L, plan.Lc
    dev = p_dev.device
    for f in range(s["n_facets"]):
        fi = plan.facet(f)
        rows = (fi["wy1"] - fi["wy0"]) * (fi["wx1"] - fi["wx0"])
        n = rows * Lc
        h = synth.hash32(torch.arange(n, dtype=torch.int64, device=dev), f, synth.WARM_P_SEED)
        u = h.double() / 4294967296.0 - 0.5
        p_dev[fi["poff"]:fi["poff"] + n] = (synth.warm_p_scale(mu_bar[f], rows) * u).float()
    I = s["n_coef"]
    pos = torch.arange(L, dtype=torch.int64, device=dev)
    scale = torch.tensor([synth.warm_w_scale(mu[p // Lc]) for p in range(L)], dtype=torch.float64, device=dev)
    wv = w_dev.view(I, L)
    for r0 in range(0, I, chunk_rows):
        r1 = min(I, r0 + chunk_rows)
        rows = torch.arange(r0, r1, dtype=torch.int64, device=dev)
        h = synth.hash32(rows[:, None], pos[None, :], synth.WARM_W_SEED)
        wv[r0:r1] = (scale[None, :] * (h.double() / 4294967296.0 - 0.5)).float()


def warm_oracle_inputs(geom, C, L, mu, mu_bar):
    """The same warm duals as callables for oracle.blocks.block_step."""
    Lc = L // C
    shapes = sara.band_shapes(geom.ny, geom.nx, geom.levels)
    offs = np.concatenate([[0], np.cumsum([a * b for a, b in shapes])]).astype(np.int64)

    def P0(c, f):
        n = f.n_rows * Lc
        return synth.warm_p_np(c * geom.Q + f.index, n, synth.warm_p_scale(mu_bar[c][f.index], f.n_rows)) \
            .reshape(f.nuc_shape + (Lc,))

    def W0(rr, cc, k, c):
        i = offs[k] + rr.astype(np.int64) * shapes[k][1] + cc
        pos = c * Lc + np.arange(Lc, dtype=np.int64)
        return synth.warm_w_np(i[..., None], pos, synth.warm_w_scale(mu[c]))

    return P0, W0


def random_weight_inputs(geom, C, theta_full, theta_bar_full):
    """Callables giving the full problem's weights (theta [C][I], theta_bar
    [C*Q] arrays) at block positions, for oracle.blocks.block_step."""
    shapes = sara.band_shapes(geom.ny, geom.nx, geom.levels)
    offs = np.concatenate([[0], np.cumsum([a * b for a, b in shapes])]).astype(np.int64)
    th = np.asarray(theta_full).reshape(C, -1)

    def theta(rr, cc, k, c):
        return th[c][offs[k] + rr.astype(np.int64) * shapes[k][1] + cc]

    def theta_bar(c, f):
        return theta_bar_full[c * geom.Q + f.index]

    return theta, theta_bar


def device_block_outputs(plan, p_dev, w_dev, g_dev, geom, blk):
    """The device results a sampled block determines: P+ of its facets
    ({(c, q): array}), W+ over the coefficient rectangles its facets own (per
    band, (rows, cols, L)), G over its exact tiles (rows, cols, L)."""
    from oracle import blocks
    C, L, Lc = plan.C, plan.L, plan.Lc
    P = {}
    for f in blk.facets(geom):
        for c in range(C):
            fi = plan.facet(c * geom.Q + f.index)
            n = (fi["wy1"] - fi["wy0"]) * (fi["wx1"] - fi["wx0"]) * Lc
            P[(c, f.index)] = p_dev[fi["poff"]:fi["poff"] + n].cpu().numpy().reshape(f.nuc_shape + (Lc,))
    bands = plan.bands()
    assert [(r, c) for r, c, _, _ in bands] == sara.band_shapes(geom.ny, geom.nx, geom.levels)
    I = plan.sizes["n_coef"]
    wv = w_dev.view(I, L)
    W = []
    for k, ((r0, r1), (c0, c1)) in enumerate(blocks.owned_rects(geom, blk)):
        rows, cols, off, _ = bands[k]
        W.append(wv[off:off + rows * cols].view(rows, cols, L)[r0:r1, c0:c1].cpu().numpy())
    (gy0, gy1), (gx0, gx1) = blocks.exact_tile_rect(geom, blk)
    G = g_dev.view(geom.ny, geom.nx, L)[gy0:gy1, gx0:gx1].cpu().numpy()
    return dict(P=P, W=W, G=G)


def block_errors(got, ref):
    """rel_l2 and max_rel of P+, W+, G between device and oracle block results."""
    keys = sorted(ref["P"])
    pairs = {
        "P": (np.concatenate([got["P"][k].reshape(-1) for k in keys]),
              np.concatenate([ref["P"][k].reshape(-1) for k in keys])),
        "W": (np.concatenate([g.reshape(-1) for g in got["W"]]), np.concatenate([r.reshape(-1) for r in ref["W"]])),
        "G": (got["G"].reshape(-1), ref["G"].reshape(-1)),
    }
    return {k: (rel_l2(a, b), max_rel(a, b), b.size) for k, (a, b) in pairs.items()}
