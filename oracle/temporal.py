"""Oracle of the temporal-stability parts of the method -- TEST INFRASTRUCTURE.

* Eq. 2, the perturbation loss, with its per-pixel term only:
  L(y, y~) = alpha * mean |y - y~| (the perceptual VGG-19 term is out of
  scope).  For each sample, x_0 is the network output on the unperturbed
  input, x_1..x_p the outputs on perturbed inputs and x~ the target:
      loss = L(x_0, x~) + sum_i L(x_0, x_i),
  with the gradient taken through x_0 only (x_1..x_p are constants).  The
  mean runs over all N*H*W pixels of the batch; the subgradient of |u| at
  u = 0 is taken as 0.
* Eq. 3, the temporal-instability metric,
      E = (1/P) sum_{p,t} [exp(alpha D_t(p)) - 1],  D_t(p) = |I_t(p) - I_{t-1}(m(p))|,
  alpha = 3.  The per-pixel part (motion-compensated lookup m(p), depth and
  normal rejection) is ``ora_temporal`` in nsm_oracle.c; rejected pixels
  contribute no term.  P is read as the total pixel count of the compared
  frames, W * H * (T - 1).  The rejection thresholds are not given in the
  paper: 1% relative view depth and a normal cosine of 0.9.
"""
import numpy as np

from . import _p, frame_vector, lib

DEPTH_TOL = 0.01
COS_TOL = 0.9


def perturbation_loss(vis, target, alpha=0.9):
    """vis [N, 1+p, H, W] (x_0 first), target [N, H, W] -> (loss, dL/dx_0 [N, H, W])."""
    v = np.asarray(vis, np.float64)
    t = np.asarray(target, np.float64)
    if v.ndim == 3:
        v, t = v[None], t[None]
    x0 = v[:, 0]
    npx = x0.size
    loss = alpha * np.abs(x0 - t).sum() / npx
    grad = np.sign(x0 - t)
    for i in range(1, v.shape[1]):
        loss += alpha * np.abs(x0 - v[:, i]).sum() / npx
        grad = grad + np.sign(x0 - v[:, i])
    return float(loss), (alpha / npx) * grad


def temporal_pair(scene, fr_prev, fr_cur, gbuf_prev, gbuf_cur, vis_prev, vis_cur, alpha=3.0,
                  depth_tol=DEPTH_TOL, cos_tol=COS_TOL):
    """One frame pair of Eq. 3 -> (sum of exp(alpha D) - 1, passed pixels, D map).

    The D map holds D(p) where the pixel passed and a negative code where it
    did not: -1 background, -2 off-screen, -3 empty previous pixel,
    -4 depth, -5 normal."""
    h, w = fr_cur.height, fr_cur.width
    tris = np.ascontiguousarray(scene.tris, np.float32)
    nrm = np.ascontiguousarray(scene.normals, np.float32)
    fa, fb = frame_vector(fr_prev), frame_vector(fr_cur)
    ga = np.ascontiguousarray(gbuf_prev, np.uint64)
    gb = np.ascontiguousarray(gbuf_cur, np.uint64)
    va = np.ascontiguousarray(vis_prev, np.float32)
    vb = np.ascontiguousarray(vis_cur, np.float32)
    total = np.zeros(1, np.float64)
    valid = np.zeros(1, np.int64)
    dmap = np.empty((h, w), np.float32)
    rc = lib().ora_temporal(_p(tris), _p(nrm), int(tris.shape[0]), _p(fa), _p(fb), _p(ga), _p(gb),
                            _p(va), _p(vb), w, h, float(alpha), float(depth_tol), float(cos_tol),
                            _p(total), _p(valid), _p(dmap))
    if rc:
        raise RuntimeError(f"ora_temporal failed ({rc})")
    return float(total[0]), int(valid[0]), dmap


def instability(sums, width, height):
    """E of Eq. 3 for a sequence from its per-pair sums (T - 1 of them)."""
    return float(np.sum(sums)) / (width * height * len(sums))
