"""Synthetic scenes, cameras and lights standing in for the paper's scenes.

The paper measures on Bistro, Sponza, Conference and Living Room at
2k x 1k (Sec. 5).  None of those assets is available, so seeded scenes of
boxes and UV-spheres on a ground quad stand in for them: the same pixel
count class (1080p), one light with a single shadow map (Sec. 1: vanilla
shadow mapping, no cascades), and screen-space feature channels.

Everything here is input generation: geometry is produced in float64 and
rounded to float32 once; camera and light matrices are built in float64 and
rounded to float32.  Matrices are row-major and map world positions to clip
space with depth range [0, 1]:

    x_clip = (p - eye).right / tan_x
    y_clip = (p - eye).up    / tan_y
    z_clip = A * zv + B,  A = far / (far - near),  B = -near * far / (far - near)
    w_clip = zv = (p - eye).fwd
"""
from dataclasses import dataclass, field
import math

import numpy as np

from .rng import SplitMix64

# Named workloads (sizes follow the paper's 2k x 1k regime and the
# tiny/batched cases used for parity).
WORKLOADS = {
    "tiny_64": dict(width=64, height=64, sm_size=128, scene="tiny"),
    "hard_1080p": dict(width=1920, height=1080, sm_size=2048, scene="objects60"),
    "soft_train_512": dict(width=512, height=512, sm_size=1024, scene="objects60",
                           windows=8, frames=4),
    "batched_mixed": dict(sizes=((1280, 720), (1920, 1080), (2560, 1440)),
                          sm_size=2048, frames=16),
}


@dataclass
class Scene:
    tris: np.ndarray      # float32 [T, 3, 3]  (triangle, vertex, xyz)
    normals: np.ndarray   # float32 [T, 3]     unit face normals (float64 -> float32)

    @property
    def n_tris(self):
        return int(self.tris.shape[0])


@dataclass
class FrameParams:
    """Per-frame light and camera parameters (all float32 except sizes)."""
    m_light: np.ndarray                 # [4, 4] row-major world -> light clip
    light_pos: np.ndarray               # [3]
    light_radius: float                 # r_e; 0 = point light
    light_near: float
    light_far: float
    light_tan_half_fov: float
    sm_size: int
    m_cam: np.ndarray                   # [4, 4] row-major world -> camera clip
    cam_pos: np.ndarray                 # [3]
    cam_fwd: np.ndarray                 # [3]
    cam_right: np.ndarray               # [3]
    cam_up: np.ndarray                  # [3]
    cam_tan_half_x: float
    cam_tan_half_y: float
    cam_near: float
    cam_far: float
    width: int
    height: int
    extra: dict = field(default_factory=dict)


# ----------------------------------------------------------------- geometry
def _face_normals(tris64):
    e1 = tris64[:, 1] - tris64[:, 0]
    e2 = tris64[:, 2] - tris64[:, 0]
    n = np.cross(e1, e2)
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def _orient_outward(tris, centre):
    """Swap vertices 1 and 2 where the winding normal points inward."""
    n = _face_normals(tris)
    c = tris.mean(axis=1) - centre
    flip = (n * c).sum(axis=1) < 0
    t = tris.copy()
    t[flip, 1], t[flip, 2] = tris[flip, 2], tris[flip, 1]
    return t


def box_tris(centre, half):
    centre = np.asarray(centre, np.float64)
    half = np.asarray(half, np.float64)
    tris = []
    for a in range(3):
        u, v = (a + 1) % 3, (a + 2) % 3
        for s in (-1.0, 1.0):
            fc = centre.copy()
            fc[a] += s * half[a]
            q = []
            for su, sv in ((-1, -1), (1, -1), (1, 1), (-1, 1)):
                p = fc.copy()
                p[u] += su * half[u]
                p[v] += sv * half[v]
                q.append(p)
            tris.append([q[0], q[1], q[2]])
            tris.append([q[0], q[2], q[3]])
    return _orient_outward(np.array(tris), centre)


_SPHERE_TEMPLATES = {}


def _unit_sphere(slices, stacks):
    """Unit-sphere directions per triangle vertex, outward-oriented (cached)."""
    key = (slices, stacks)
    if key not in _SPHERE_TEMPLATES:
        def vert(i, j):
            th = math.pi * i / stacks
            ph = 2.0 * math.pi * (j % slices) / slices
            return np.array([math.sin(th) * math.cos(ph), math.cos(th), math.sin(th) * math.sin(ph)])

        tris = []
        for j in range(slices):
            tris.append([vert(0, 0), vert(1, j), vert(1, j + 1)])
            tris.append([vert(stacks, 0), vert(stacks - 1, j + 1), vert(stacks - 1, j)])
        for i in range(1, stacks - 1):
            for j in range(slices):
                a, b = vert(i, j), vert(i, j + 1)
                c, d = vert(i + 1, j), vert(i + 1, j + 1)
                tris.append([a, c, d])
                tris.append([a, d, b])
        _SPHERE_TEMPLATES[key] = _orient_outward(np.array(tris), np.zeros(3))
    return _SPHERE_TEMPLATES[key]


def uv_sphere_tris(centre, radius, slices=20, stacks=17):
    """UV sphere: two pole fans plus (stacks - 2) quad bands, outward winding."""
    centre = np.asarray(centre, np.float64)
    return centre + radius * _unit_sphere(slices, stacks)


def ground_quad(y=-1.0, half=1.5, cells=1):
    """Ground plane y = const over [-half, half]^2, split into cells x cells quads."""
    tris = []
    xs = np.linspace(-half, half, cells + 1)
    for i in range(cells):
        for k in range(cells):
            p00 = np.array([xs[i], y, xs[k]])
            p10 = np.array([xs[i + 1], y, xs[k]])
            p11 = np.array([xs[i + 1], y, xs[k + 1]])
            p01 = np.array([xs[i], y, xs[k + 1]])
            tris.append([p00, p01, p11])
            tris.append([p00, p11, p10])
    return np.array(tris)


def _finish(tri_list):
    t64 = np.concatenate(tri_list, axis=0)
    t32 = t64.astype(np.float32)
    n = _face_normals(t32.astype(np.float64)).astype(np.float32)
    return Scene(tris=np.ascontiguousarray(t32), normals=np.ascontiguousarray(n))


def make_scene(kind, seed, n_spheres=30, n_boxes=30, stacks=17, slices=20):
    """Seeded scene.

    ``tiny``: ground quad y = -1 over [-1.5, 1.5]^2 plus 4 boxes with centres
    U[-1, 1]^3 and half-extents U[0.1, 0.5]^3 (50 triangles).

    ``objects60``: a ground plane y = -1 over [-3, 3]^2 (6 x 6 quads, 72
    triangles) plus ``n_boxes`` boxes (half-extents U[0.03, 0.15]^3) and
    ``n_spheres`` UV-spheres (radius U[0.03, 0.15]), centres
    U[-1, 1] x U[-1, -0.5] x U[-1, 1]; 30 + 30 with 20 x 17 spheres gives
    19,632 triangles.
    """
    rng = SplitMix64(seed).fork(0x5CE7E)
    if kind == "tiny":
        parts = [ground_quad()]
    else:
        parts = [ground_quad(half=3.0, cells=6)]
    if kind == "tiny":
        for _ in range(4):
            c = rng.uniforms(3, -1.0, 1.0)
            h = rng.uniforms(3, 0.1, 0.5)
            parts.append(box_tris(c, h))
    elif kind == "objects60":
        for _ in range(n_boxes):
            c = np.array([rng.uniform(-1, 1), rng.uniform(-1, -0.5), rng.uniform(-1, 1)])
            h = rng.uniforms(3, 0.03, 0.15)
            parts.append(box_tris(c, h))
        for _ in range(n_spheres):
            c = np.array([rng.uniform(-1, 1), rng.uniform(-1, -0.5), rng.uniform(-1, 1)])
            r = rng.uniform(0.03, 0.15)
            parts.append(uv_sphere_tris(c, r, slices=slices, stacks=stacks))
    else:
        raise ValueError(f"unknown scene kind {kind!r}")
    return _finish(parts)


# ------------------------------------------------------- cameras and lights
def _basis(eye, target, ref_up):
    fwd = target - eye
    fwd = fwd / np.linalg.norm(fwd)
    if abs(float(np.dot(fwd, ref_up))) > 0.95:
        ref_up = np.array([0.0, 0.0, 1.0]) if abs(fwd[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    right = np.cross(fwd, ref_up)
    right = right / np.linalg.norm(right)
    up = np.cross(right, fwd)
    return fwd, right, up


def _matrix(eye, fwd, right, up, tan_x, tan_y, near, far):
    A = far / (far - near)
    B = -near * far / (far - near)
    m = np.zeros((4, 4))
    m[0, :3] = right / tan_x
    m[0, 3] = -np.dot(right, eye) / tan_x
    m[1, :3] = up / tan_y
    m[1, 3] = -np.dot(up, eye) / tan_y
    m[2, :3] = fwd * A
    m[2, 3] = -np.dot(fwd, eye) * A + B
    m[3, :3] = fwd
    m[3, 3] = -np.dot(fwd, eye)
    return m


def _view_coords(pts, eye, fwd, right, up):
    d = pts - eye
    return d @ right, d @ up, d @ fwd


def make_frame(scene, width, height, sm_size, light_pos, eye, target=(0.0, 0.0, 0.0),
               vfov_deg=50.0, light_radius=0.0):
    """Camera and light parameters for one frame.

    The light frustum is square, looks at the centre of the scene's bounding
    box and is fitted to every vertex (so the whole scene is inside the
    shadow map); the camera near/far planes are fitted to the vertices in
    front of it.
    """
    pts = scene.tris.reshape(-1, 3).astype(np.float64)
    lo, hi = pts.min(0), pts.max(0)
    centre = 0.5 * (lo + hi)
    L = np.asarray(light_pos, np.float64)
    fwd, right, up = _basis(L, centre, np.array([0.0, 0.0, 1.0]))
    xv, yv, zv = _view_coords(pts, L, fwd, right, up)
    if zv.min() <= 1e-3:
        raise ValueError("scene is not entirely in front of the light")
    tan_l = float(np.max(np.maximum(np.abs(xv), np.abs(yv)) / zv)) * 1.02
    near_l = float(zv.min()) * 0.95
    far_l = float(zv.max()) * 1.05
    m_light = _matrix(L, fwd, right, up, tan_l, tan_l, near_l, far_l)

    E = np.asarray(eye, np.float64)
    cf, cr, cu = _basis(E, np.asarray(target, np.float64), np.array([0.0, 1.0, 0.0]))
    tan_y = math.tan(math.radians(vfov_deg) * 0.5)
    tan_x = tan_y * width / height
    _, _, czv = _view_coords(pts, E, cf, cr, cu)
    if czv.min() <= 0.05:
        raise ValueError("scene geometry behind the camera near plane")
    near_c = float(czv.min()) * 0.9
    far_c = float(czv.max()) * 1.1
    m_cam = _matrix(E, cf, cr, cu, tan_x, tan_y, near_c, far_c)

    f32 = np.float32
    return FrameParams(
        m_light=m_light.astype(f32), light_pos=L.astype(f32), light_radius=float(f32(light_radius)),
        light_near=float(f32(near_l)), light_far=float(f32(far_l)),
        light_tan_half_fov=float(f32(tan_l)), sm_size=int(sm_size),
        m_cam=m_cam.astype(f32), cam_pos=E.astype(f32), cam_fwd=cf.astype(f32),
        cam_right=cr.astype(f32), cam_up=cu.astype(f32),
        cam_tan_half_x=float(f32(tan_x)), cam_tan_half_y=float(f32(tan_y)),
        cam_near=float(f32(near_c)), cam_far=float(f32(far_c)),
        width=int(width), height=int(height))


def _eye_on_ring(rng, radius=3.0, height=1.5):
    phi = rng.uniform(0.0, 2.0 * math.pi)
    return np.array([radius * math.cos(phi), height, radius * math.sin(phi)])


# Camera aim for the object scenes: a point on the ground so that the ground
# plane fills most of a 16:9 view (about 70% foreground pixels).
GROUND_TARGET = (0.0, -1.0, 0.0)


def workload_frame(name, seed):
    """(scene, frame) for the single-frame named workloads."""
    w = WORKLOADS[name]
    scene = make_scene(w["scene"], seed)
    rng = SplitMix64(seed).fork(0x11647)
    if w["scene"] == "tiny":
        light = np.array([rng.uniform(-1, 1), rng.uniform(2, 3), rng.uniform(-1, 1)])
        eye, target = _eye_on_ring(rng), (0.0, 0.0, 0.0)
    else:
        light = np.array([rng.uniform(-1, 1), rng.uniform(2.5, 4), rng.uniform(-1, 1)])
        eye, target = _eye_on_ring(rng, radius=3.2, height=1.5), GROUND_TARGET
    return scene, make_frame(scene, w["width"], w["height"], w["sm_size"], light, eye, target=target)


def _catmull_rom(p, u):
    p0, p1, p2, p3 = p
    return 0.5 * ((2 * p1) + (-p0 + p2) * u + (2 * p0 - 5 * p1 + 4 * p2 - p3) * u * u
                  + (-p0 + 3 * p1 - 3 * p2 + p3) * u * u * u)


def make_train_window(seed, window, frames=4, width=512, height=512, sm_size=1024, scene=None):
    """One temporal window: camera and spherical light on Catmull-Rom splines.

    Four seed control points per spline; consecutive frames are 1/60 of the
    spline parameter apart; light radius r_e ~ U[0.02, 0.2].
    """
    if scene is None:
        scene = make_scene("objects60", seed)
    rng = SplitMix64(seed).fork(0x7A1 + 97 * window)
    phi0 = rng.uniform(0, 2 * math.pi)
    dphi = rng.uniform(0.1, 0.3)
    cam_pts = []
    for k in range(4):
        r = rng.uniform(2.9, 3.5)
        h = rng.uniform(1.3, 1.8)
        ph = phi0 + k * dphi
        cam_pts.append(np.array([r * math.cos(ph), h, r * math.sin(ph)]))
    light_pts = [np.array([rng.uniform(-1, 1), rng.uniform(2.5, 4), rng.uniform(-1, 1)])
                 for _ in range(4)]
    radius = rng.uniform(0.02, 0.2)
    u0 = rng.uniform(0.0, 1.0 - (frames - 1) / 60.0)
    out = []
    for k in range(frames):
        u = u0 + k / 60.0
        fr = make_frame(scene, width, height, sm_size, _catmull_rom(light_pts, u),
                        _catmull_rom(cam_pts, u), target=GROUND_TARGET, light_radius=radius)
        out.append(fr)
    return scene, out


def perturb_frame(scene, fr, seed, cam_scale=0.004, light_scale=0.004, size_scale=0.5):
    """A jittered copy of a frame, the input of one perturbed network
    instance of the perturbation loss (Sec. 3.3): the camera and the emitter
    move by small random offsets that grow with their distance from the
    scene and, for the emitter, with its size.

    Offsets are uniform in a ball of radius cam_scale * |eye - c| for the
    camera (keeping its aim point) and light_scale * |L - c| + size_scale *
    r_e for the emitter, c the centre of the scene's bounding box.  The
    scales are not given in the paper."""
    rng = SplitMix64(seed).fork(0x9E27)
    pts = scene.tris.reshape(-1, 3).astype(np.float64)
    c = 0.5 * (pts.min(0) + pts.max(0))

    def ball(radius):
        while True:
            v = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-1, 1)])
            if v @ v <= 1.0:
                return radius * v

    eye = fr.cam_pos.astype(np.float64)
    target = eye + 3.0 * fr.cam_fwd.astype(np.float64)
    L = fr.light_pos.astype(np.float64)
    eye2 = eye + ball(cam_scale * np.linalg.norm(eye - c))
    L2 = L + ball(light_scale * np.linalg.norm(L - c) + size_scale * fr.light_radius)
    vfov = 2.0 * math.degrees(math.atan(fr.cam_tan_half_y))
    return make_frame(scene, fr.width, fr.height, fr.sm_size, L2, eye2, target=target, vfov_deg=vfov,
                      light_radius=fr.light_radius)


def make_batched_frames(seed, n_frames=16, sizes=((1280, 720), (1920, 1080), (2560, 1440)),
                        sm_size=2048):
    """Mixed-size frames from scenes of ~20k-100k triangles, hard and soft lights."""
    rng = SplitMix64(seed).fork(0xBA7C)
    frames = []
    for f in range(n_frames):
        n_sph = int(30 + rng.uniform(0, 1) * 120)
        scene = make_scene("objects60", seed * 1000 + f, n_spheres=n_sph)
        w, h = sizes[int(rng.uniform(0, len(sizes))) % len(sizes)]
        light = np.array([rng.uniform(-1, 1), rng.uniform(2.5, 4), rng.uniform(-1, 1)])
        radius = 0.0 if rng.uniform() < 0.5 else rng.uniform(0.02, 0.2)
        frames.append((scene, make_frame(scene, w, h, sm_size, light,
                                         _eye_on_ring(rng, radius=3.2, height=1.5),
                                         target=GROUND_TARGET, light_radius=radius)))
    return frames
