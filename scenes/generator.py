"""Seeded synthetic scenes standing in for the photo collections of Table 3.

Every camera is a pinhole with f = 1000 px, a 1024 x 768 image, principal
point (512, 384), x to the right and y down, looking at the scene centre.
World points project as x ~ K (R X + t).

Descriptor model (per 3D point one base vector, per view a noisy copy):
  base  = clip(rint(|N(0, 30)|), 0, 127), iid over 128 dimensions
  view  = clip(base + U{-6..6}, 0, 127)
Distractor features get a fresh base vector plus view noise and a uniform
position in the image.  Keypoints of true features are the projection plus
N(0, 0.5 px) per coordinate; a feature is kept when its point is in front of
the camera and its noisy keypoint is inside the image.  The order of the
features in every image is a seeded random permutation.

The fundamental matrix of a pair follows Section 6.2 eq. (1) written in the
library convention x_b^T F x_a = 0 (line in image b is F x_a): with world to
camera poses (R_a, t_a), (R_b, t_b),
  R = R_b R_a^T,  t = t_b - R t_a,  F = K_b^{-T} [t]_x R K_a^{-1}.
This is input preparation: the matcher receives F and never builds it.
"""
from __future__ import annotations

import threading
from dataclasses import dataclass, field

import numpy as np

IMG_W = 1024
IMG_H = 768
FOCAL = 1000.0
PRINCIPAL = (512.0, 384.0)
DESC_DIM = 128

# numpy's BLAS gives wrong results when several threads call it at once, so
# the matrix products that image generation makes run one at a time.
_BLAS_LOCK = threading.Lock()


@dataclass
class Camera:
    K: np.ndarray      # 3x3 intrinsics
    R: np.ndarray      # world -> camera rotation
    t: np.ndarray      # x_cam = R X + t

    @property
    def center(self) -> np.ndarray:
        with _BLAS_LOCK:
            return -self.R.T @ self.t


@dataclass
class Image:
    xy: np.ndarray     # float32 (n, 2), pixel coordinates
    desc: np.ndarray   # uint8 (n, 128), values 0..127
    gt: np.ndarray     # int32 (n,), 3D point id or -1 for a distractor
    scale: np.ndarray = None   # float32 (n,): the feature's scale (multi-view scenes)

    @property
    def n(self) -> int:
        return int(self.xy.shape[0])


def intrinsics() -> np.ndarray:
    return np.array([[FOCAL, 0.0, PRINCIPAL[0]],
                     [0.0, FOCAL, PRINCIPAL[1]],
                     [0.0, 0.0, 1.0]])


def look_at_camera(center, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)) -> Camera:
    """Camera at `center` whose optical axis points at `target` (y down)."""
    c = np.asarray(center, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - c
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, dtype=np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    return Camera(intrinsics(), R, -R @ c)


def project(cam: Camera, X: np.ndarray):
    """Pixel coordinates and camera depth of world points X (n, 3)."""
    with _BLAS_LOCK:
        Xc = X @ cam.R.T + cam.t
        uvw = Xc @ cam.K.T
    with np.errstate(divide="ignore", invalid="ignore"):
        xy = uvw[:, :2] / uvw[:, 2:3]
    return xy, Xc[:, 2]


def skew(v) -> np.ndarray:
    x, y, z = v
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def fundamental_from_poses(cam_a: Camera, cam_b: Camera) -> np.ndarray:
    """F with x_b^T F x_a = 0 (Section 6.2 eq. 1 in the a -> b direction)."""
    R = cam_b.R @ cam_a.R.T
    t = cam_b.t - R @ cam_a.t
    E = skew(t) @ R
    return np.linalg.inv(cam_b.K).T @ E @ np.linalg.inv(cam_a.K)


def base_descriptors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = np.rint(np.abs(rng.normal(0.0, 30.0, size=(n, DESC_DIM))))
    return np.clip(v, 0, 127).astype(np.uint8)


def view_descriptors(rng: np.random.Generator, base: np.ndarray) -> np.ndarray:
    noise = rng.integers(-6, 7, size=base.shape, dtype=np.int16)
    return np.clip(base.astype(np.int16) + noise, 0, 127).astype(np.uint8)


def _inside(xy: np.ndarray) -> np.ndarray:
    return ((xy[:, 0] >= 0.0) & (xy[:, 0] < IMG_W)
            & (xy[:, 1] >= 0.0) & (xy[:, 1] < IMG_H))


def _assemble_image(rng, cam, X, base, cand_ids, n_features, n_true_max):
    """Noisy keypoints for the visible candidates, distractors to fill, shuffle.

    cand_ids are tried in the given order; the first n_true_max that stay
    inside the image after keypoint noise become true features.
    """
    xy_p, z = project(cam, X[cand_ids])
    noisy = xy_p + rng.normal(0.0, 0.5, size=xy_p.shape)
    keep = (z > 0) & _inside(noisy)
    ids = cand_ids[keep][:n_true_max]
    xy_true = noisy[keep][:n_true_max]
    n_true = ids.shape[0]
    n_dis = max(0, n_features - n_true)
    xy_dis = np.stack([rng.uniform(0.0, IMG_W, n_dis),
                       rng.uniform(0.0, IMG_H, n_dis)], axis=1)
    desc_true = view_descriptors(rng, base[ids])
    desc_dis = view_descriptors(rng, base_descriptors(rng, n_dis))
    xy = np.concatenate([xy_true, xy_dis]).astype(np.float32)
    # float32 rounding can push a coordinate onto the far image edge
    xy[:, 0] = np.minimum(xy[:, 0], np.float32(np.nextafter(np.float32(IMG_W), 0)))
    xy[:, 1] = np.minimum(xy[:, 1], np.float32(np.nextafter(np.float32(IMG_H), 0)))
    desc = np.concatenate([desc_true, desc_dis])
    gt = np.concatenate([ids.astype(np.int32), np.full(n_dis, -1, np.int32)])
    perm = rng.permutation(xy.shape[0])
    return Image(np.ascontiguousarray(xy[perm]), np.ascontiguousarray(desc[perm]),
                 np.ascontiguousarray(gt[perm]))


# ----------------------------------------------------------------------------
# Two-view scenes (one pair)
# ----------------------------------------------------------------------------

@dataclass
class PairScene:
    cams: list
    images: list
    points: np.ndarray
    F: np.ndarray          # (3, 3), x_1^T F x_0 = 0
    band_px: float

    @property
    def pairs(self):
        return [(0, 1, self.band_px)]


def make_pair_scene(n_points: int, n_features: int, sep_deg: float = 15.0,
                    radius: float = 20.0, box: float = 5.0, band_px: float = 4.0,
                    seed: int = 0) -> PairScene:
    """Points uniform in [-box, box]^3, two cameras on a horizontal circle."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-box, box, size=(n_points, 3))
    base = base_descriptors(rng, n_points)
    half = np.deg2rad(sep_deg) / 2.0
    cams = [look_at_camera((radius * np.sin(th), 0.0, radius * np.cos(th)))
            for th in (-half, half)]
    ids = np.arange(n_points)
    images = [_assemble_image(rng, cam, X, base, ids, n_features, n_features)
              for cam in cams]
    return PairScene(cams, images, X, fundamental_from_poses(cams[0], cams[1]),
                     band_px)


def make_two_view_2k(seed: int = 0) -> PairScene:
    """One pair: 1,500 points, 2 cameras 15 deg apart, 2,000 features each."""
    return make_pair_scene(1500, 2000, seed=seed)


def make_two_view_16k(seed: int = 0) -> PairScene:
    """One large pair: 16,000 features per image, about 40% true (6,400 points)."""
    return make_pair_scene(6400, 16000, seed=seed)


# ----------------------------------------------------------------------------
# Multi-view scenes with covisibility structure
# ----------------------------------------------------------------------------

@dataclass
class MultiViewScene:
    cams: list
    points: np.ndarray         # (m, 3)
    normals: np.ndarray        # (m, 3) unit
    base: np.ndarray           # (m, 128) uint8
    saliency: np.ndarray       # (m,) global per-point order of preference
    n_features: np.ndarray     # (n_images,) feature count per image
    true_frac: float
    cone_deg: float
    seed: int
    _cache: dict = field(default_factory=dict, repr=False)

    @property
    def n_images(self) -> int:
        return len(self.cams)

    def visible_ids(self, i: int) -> np.ndarray:
        """Points in front of camera i, inside its image and inside their cone."""
        cam = self.cams[i]
        xy, z = project(cam, self.points)
        v = self.cams[i].center[None, :] - self.points
        dist = np.linalg.norm(v, axis=1)
        cone = np.einsum("ij,ij->i", v, self.normals) >= np.cos(np.deg2rad(self.cone_deg)) * dist
        return np.nonzero((z > 0) & _inside(xy) & cone)[0]

    def image(self, i: int) -> Image:
        if i in self._cache:
            return self._cache[i]
        rng = np.random.default_rng([self.seed, 7, i])
        vis = self.visible_ids(i)
        order = vis[np.argsort(-self.saliency[vis], kind="stable")]
        n = int(self.n_features[i])
        n_true = int(round(self.true_frac * n))
        img = _assemble_image(rng, self.cams[i], self.points, self.base, order, n, n_true)
        # Scale: a true feature takes its point's saliency (the images keep their
        # most salient visible points, so large scales repeat across views, as
        # high-scale SIFT does); a distractor a uniform draw of its own.
        srng = np.random.default_rng([self.seed, 11, i])
        scale = srng.uniform(0.0, 1.0, size=img.gt.shape[0])
        true = img.gt >= 0
        scale[true] = self.saliency[img.gt[true]]
        img.scale = scale.astype(np.float32)
        self._cache[i] = img
        return img

    def F(self, a: int, b: int) -> np.ndarray:
        return fundamental_from_poses(self.cams[a], self.cams[b])


def by_scale(img: Image) -> Image:
    """The image with its features listed in decreasing scale (ties keep their
    order), the order a feature extractor emits them in."""
    order = np.argsort(-img.scale, kind="stable")
    return Image(img.xy[order], img.desc[order], img.gt[order], img.scale[order])


def make_multiview_scene(cam_centers, n_lo: int, n_hi: int, n_points: int = 200_000,
                         box: float = 5.0, true_frac: float = 0.6,
                         cone_deg: float = 75.0, seed: int = 0) -> MultiViewScene:
    rng = np.random.default_rng([seed, 1])
    X = rng.uniform(-box, box, size=(n_points, 3))
    nrm = rng.normal(size=(n_points, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    base = base_descriptors(rng, n_points)
    saliency = rng.uniform(size=n_points)
    cams = [look_at_camera(c) for c in cam_centers]
    nf = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=len(cams)))).astype(np.int64)
    return MultiViewScene(cams, X, nrm, base, saliency, nf, true_frac, cone_deg, seed)


def _ring(n: int, radius: float, elev_deg: float, az0: float = 0.0, span: float = 360.0,
          endpoint: bool = False):
    az = np.deg2rad(az0 + np.linspace(0.0, span, n, endpoint=endpoint))
    el = np.deg2rad(elev_deg)
    return [(radius * np.cos(el) * np.sin(a), radius * np.sin(el), radius * np.cos(el) * np.cos(a))
            for a in az]


def make_arc_batch(seed: int = 0):
    """60 cameras on a 180 deg arc (radius 20), 2k-20k features, 500 pairs 5-30 deg apart."""
    centers = _ring(60, 20.0, 0.0, az0=-90.0, span=180.0, endpoint=True)
    scene = make_multiview_scene(centers, 2000, 20000, seed=seed)
    az = np.linspace(-90.0, 90.0, 60)
    pairs = sample_pairs_by_angle(az, 5.0, 30.0, 500, seed=1)
    return scene, [(a, b, 4.0) for a, b in pairs]


def make_three_rings(seed: int = 0):
    """300 cameras on 3 rings x 100 (elevations -15/0/+15), 4k-25k features."""
    centers = []
    for el in (-15.0, 0.0, 15.0):
        centers += _ring(100, 20.0, el)
    return make_multiview_scene(centers, 4000, 25000, seed=seed)


def make_ten_rings(seed: int = 0):
    """1,000 cameras on 10 rings x 100 (elevations -30..+30, radii 18-26), 8k-40k features."""
    centers = []
    for el, r in zip(np.linspace(-30.0, 30.0, 10), np.linspace(18.0, 26.0, 10)):
        centers += _ring(100, float(r), float(el))
    return make_multiview_scene(centers, 8000, 40000, seed=seed)


def sample_pairs_by_angle(az_deg, lo: float, hi: float, n: int, seed: int = 1):
    """n ordered pairs (a, b), a != b, whose azimuths differ by lo..hi degrees."""
    az = np.asarray(az_deg)
    cand = [(a, b) for a in range(len(az)) for b in range(len(az))
            if a != b and lo <= abs(az[a] - az[b]) <= hi]
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(cand), size=min(n, len(cand)), replace=False)
    return [cand[k] for k in sorted(idx)]


def covisible_pairs(scene: MultiViewScene, min_shared: int = 8, top_k: int = 30):
    """Ordered pairs (q, c) whose images share >= min_shared ground-truth points,
    keeping for every query image its top_k partners by shared count
    (the candidate-image rule of Section 6.1 on ground-truth visibility)."""
    from scipy import sparse
    rows, cols = [], []
    for i in range(scene.n_images):
        g = scene.image(i).gt
        g = np.unique(g[g >= 0])
        rows.append(np.full(g.shape[0], i))
        cols.append(g)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    V = sparse.csr_matrix((np.ones(rows.shape[0], np.int32), (rows, cols)),
                          shape=(scene.n_images, scene.points.shape[0]))
    C = (V @ V.T).toarray()
    np.fill_diagonal(C, 0)
    out = []
    for q in range(scene.n_images):
        ok = np.nonzero(C[q] >= min_shared)[0]
        ok = ok[np.argsort(-C[q, ok], kind="stable")][:top_k]
        out += [(q, int(c)) for c in sorted(ok)]
    return out


def visibility_lists(scene: MultiViewScene):
    """The coarse-model visibility: per image, the sorted ids of the 3D points
    its true features observe."""
    out = []
    for i in range(scene.n_images):
        g = scene.image(i).gt
        out.append(np.unique(g[g >= 0]).astype(np.int32))
    return out


def visibility_csr(vis_lists):
    """The lists as CSR arrays: offsets int32[n + 1] and point ids int32[nnz]."""
    off = np.zeros(len(vis_lists) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(p) for p in vis_lists])
    pts = np.concatenate([np.asarray(p, dtype=np.int32) for p in vis_lists]) \
        if len(vis_lists) else np.zeros(0, np.int32)
    return off.astype(np.int32), pts.astype(np.int32)


def materialize(scene: MultiViewScene, workers: int = 8, progress=None) -> None:
    """Generate every image of a multi-view scene into its cache with a
    thread pool.  Each image draws from its own seeded generator, so the
    bytes do not depend on the order or the number of workers."""
    from concurrent.futures import ThreadPoolExecutor
    todo = [i for i in range(scene.n_images) if i not in scene._cache]
    with ThreadPoolExecutor(max(1, int(workers))) as ex:
        for k, _ in enumerate(ex.map(scene.image, todo)):
            if progress is not None and (k + 1) % 200 == 0:
                progress(k + 1, len(todo))


def stress_requests(scene: MultiViewScene, n_requests: int = 20_000, band_lo: float = 2.0,
                    band_hi: float = 8.0, seed: int = 1):
    """Stress-serving requests: n_requests distinct covisible pairs (top 30
    per image, >= 8 shared points) in a seeded random order, each with its own
    band half-width drawn uniformly from [band_lo, band_hi] px."""
    pool = covisible_pairs(scene)
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(pool), size=min(n_requests, len(pool)), replace=False)
    bands = rng.uniform(band_lo, band_hi, size=pick.shape[0])
    return [(pool[k][0], pool[k][1], float(d)) for k, d in zip(pick, bands)]


def poisson_arrivals(rate_per_s: float, duration_s: float, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of an open-loop Poisson stream."""
    rng = np.random.default_rng(seed)
    n = int(rate_per_s * duration_s * 1.5) + 16
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
    return t[t < duration_s]
