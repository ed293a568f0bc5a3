"""Principal components before k-means (paper section 4.1, "PCA and k-means
clustering"), and the pruning built on it.  Test infrastructure only.

Section 4.1 transforms the performance vectors with principal component
analysis -- fewer coordinates, the variance concentrated in the leading
ones -- and clusters the transformed points with k-means.  Each cluster's
kernel then follows section 4.2: k-means gives a representative (the
centroid), so the kernel is the configuration best for it, read in the
original coordinates; or, from the labels alone, the configuration best for
the geometric mean of the members (``oracle.represent``).

Readings (the paper gives no formulas):

* points are the rows of the Q16 normalized table as x = q / 65535 (FP64);
* centring at the column means; covariance C = Xc^T Xc / (n - 1);
* components: unit eigenvectors of C by decreasing eigenvalue, each signed
  so that its first entry whose magnitude is within a factor 1 - 1e-9 of
  the largest is positive; explained variance of the first m components =
  their eigenvalues' sum / trace(C);
* the projection Z = Xc V_m is quantized for the integer k-means with one
  offset and one scale for every coordinate, so distances keep their
  ratios: U = rint((Z - lo) / span * 65535), lo = min Z, span = max Z - lo
  (all U = 0 when span = 0);
* a centroid c of U stands for z = lo + c * span / 65535, i.e. the point
  x = mean + V_m z in the original coordinates, read as Q16 values
  rint(65535 x); its kernel is the largest of those (section 4.2's rule for
  representatives, picks distinct as in ``oracle.represent``).
"""
from __future__ import annotations

import numpy as np

from . import kmeans as okm
from . import normalize as onorm
from . import represent as orep

REP_CENTROID, REP_GEOMEAN = 0, 1


def _sign_fix(v: np.ndarray) -> np.ndarray:
    a = np.abs(v)
    first = int(np.argmax(a >= (1.0 - 1e-9) * a.max()))
    return -v if v[first] < 0 else v


def pca(X, m: int):
    """X: n x d FP64 points (n >= 2).  Returns dict(mean, components (m x d),
    variances (all d eigenvalues, decreasing), Z (n x m), explained)."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    mean = X.mean(axis=0)
    Xc = X - mean
    C = Xc.T @ Xc / (n - 1)
    w, V = np.linalg.eigh(C)              # ascending eigenvalues, unit columns
    order = np.argsort(-w, kind="stable")
    w, V = w[order], V[:, order]
    comps = np.array([_sign_fix(V[:, i]) for i in range(d)])
    tr = float(np.trace(C))
    explained = float(w[:m].sum() / tr) if tr > 0 else 1.0
    return dict(mean=mean, components=comps[:m], variances=w, Z=Xc @ comps[:m].T,
                explained=explained)


def quantize(Z):
    """(U uint16, lo, span): one offset and scale for every coordinate."""
    Z = np.asarray(Z, dtype=np.float64)
    lo = float(Z.min())
    span = float(Z.max()) - lo
    if span == 0.0:
        return np.zeros(Z.shape, dtype=np.uint16), lo, span
    return np.rint((Z - lo) / span * 65535.0).astype(np.uint16), lo, span


def centroid_q16(c, lo: float, span: float, mean, components) -> np.ndarray:
    """A centroid of the quantized space read back as Q16 values of every
    configuration (int64, not clamped)."""
    z = lo + np.asarray(c, dtype=np.float64) * span / 65535.0
    x = np.asarray(mean) + np.asarray(components).T @ z
    return np.rint(65535.0 * x).astype(np.int64)


def prune_pca(T, k: int, norm: int, m: int, rep: int, draws_per_restart, max_iter: int = 300):
    """PCA + k-means pruning of a timing table (rows = problems): normalize
    (section 3.4), project on the first m components, quantize, integer
    k-means (``oracle.kmeans``), one kernel per cluster by ``rep``."""
    Xq = onorm.normalize(T, norm)
    P = pca(Xq.astype(np.float64) / 65535.0, m)
    U, lo, span = quantize(P["Z"])
    km = okm.kmeans(U.astype(np.int64), k, draws_per_restart, max_iter)
    if rep == REP_CENTROID:
        scores = [centroid_q16(c, lo, span, P["mean"], P["components"]) for c in km["centroids"]]
        chosen = orep.pick_distinct(scores, k)
    else:
        chosen = orep.geomean_representatives(Xq, km["labels"], k, k)
    return dict(chosen=chosen, labels=km["labels"], inertia=km["inertia"], U=U, lo=lo, span=span,
                explained=P["explained"], pca=P)
