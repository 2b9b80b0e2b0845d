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
