"""Seeded synthetic scene generator.

This module only builds inputs: triangle soups, material records, an emission
texture and a pinhole camera.  It holds none of the rendering arithmetic; the
FP64 oracle and the HIP library both read the arrays it returns.

Scene dictionary (all arrays little-endian, C-contiguous):
  tri     float32 (T, 9)   v0, v1, v2 of every triangle (flat shading; the
                            geometric normal is (v1-v0) x (v2-v0), normalised;
                            emitters emit on that side, conductors reflect only
                            on that side, dielectrics call it "outside")
  tri_mat int32   (T,)     material index
  tri_uv  float32 (T, 6)   per-vertex (u, v), used to look up the emission texture
  mats    float32 (NM, 16) material records, see MAT_* below
  tex     float32 (TH, TW) emission texture (multiplies Le when textured=1)
  cam     float32 (10,)    position(3), target(3), up(3), vertical fov in degrees
  width, height            image size in pixels

Material record layout (float32[16]):
  [0] type (MAT_LAMBERT, MAT_CONDUCTOR, MAT_DIELECTRIC)
  [1:4] albedo (Lambert) or F0 (conductor, Schlick); unused for dielectric
  [4] roughness (conductor; GGX alpha = max(roughness^2, 1e-4))
  [5] index of refraction (dielectric; the outside medium has index 1)
  [6:9] emitted radiance Le (RGB); non-zero only for Lambert materials
  [9] 1 if Le is multiplied by the emission texture at the hit's (u, v)
A vertex is specular (S) when its material is a conductor or a dielectric with
roughness below 0.2 (Section 6.1's rule); every other vertex is diffuse (D).

Random choices use numpy's Philox bit generator keyed by the config id, so the
same id always yields the same scene.
"""
import math

import numpy as np

MAT_LAMBERT = 0
MAT_CONDUCTOR = 1
MAT_DIELECTRIC = 2


def _rng(key):
    return np.random.Generator(np.random.Philox(key=int(key)))


def material(kind, rgb=(0.0, 0.0, 0.0), roughness=0.0, ior=1.5, le=(0.0, 0.0, 0.0), textured=0):
    m = np.zeros(16, np.float32)
    m[0] = kind
    m[1:4] = rgb
    m[4] = roughness
    m[5] = ior
    m[6:9] = le
    m[9] = textured
    return m


class Builder:
    """Accumulates triangles and materials."""

    def __init__(self):
        self.tris, self.mats_idx, self.uvs, self.mats = [], [], [], []

    def add_material(self, m):
        self.mats.append(np.asarray(m, np.float32))
        return len(self.mats) - 1

    def add_tris(self, tris, mat, uvs=None):
        tris = np.asarray(tris, np.float64).reshape(-1, 9)
        self.tris.append(tris)
        self.mats_idx.append(np.full(len(tris), mat, np.int32))
        if uvs is None:
            uvs = np.zeros((len(tris), 6))
        self.uvs.append(np.asarray(uvs, np.float64).reshape(-1, 6))

    def add_quad(self, p0, p1, p2, p3, mat, with_uv=False):
        """Quad p0,p1,p2,p3 (counter-clockwise seen from the front side)."""
        p0, p1, p2, p3 = (np.asarray(p, np.float64) for p in (p0, p1, p2, p3))
        tris = [np.concatenate([p0, p1, p2]), np.concatenate([p0, p2, p3])]
        uvs = None
        if with_uv:
            uvs = [[0, 0, 1, 0, 1, 1], [0, 0, 1, 1, 0, 1]]
        self.add_tris(tris, mat, uvs)

    def add_rect(self, center, half_u, half_v, normal, mat, with_uv=False):
        """Rectangle center +- half_u +- half_v whose front side faces `normal`."""
        c, a, b = (np.asarray(x, np.float64) for x in (center, half_u, half_v))
        if np.dot(np.cross(a, b), np.asarray(normal, np.float64)) < 0:
            b = -b
        self.add_quad(c - a - b, c + a - b, c + a + b, c - a + b, mat, with_uv)

    def build(self, cam, width, height, tex=None):
        tex = np.ones((1, 1), np.float32) if tex is None else np.asarray(tex, np.float32)
        return {
            "tri": np.ascontiguousarray(np.concatenate(self.tris).astype(np.float32)),
            "tri_mat": np.ascontiguousarray(np.concatenate(self.mats_idx).astype(np.int32)),
            "tri_uv": np.ascontiguousarray(np.concatenate(self.uvs).astype(np.float32)),
            "mats": np.ascontiguousarray(np.stack(self.mats).astype(np.float32)),
            "tex": np.ascontiguousarray(tex),
            "cam": np.asarray(cam, np.float32),
            "width": int(width),
            "height": int(height),
        }


# ---------------------------------------------------------------------------
# meshes
# ---------------------------------------------------------------------------

def icosphere(subdiv):
    """Unit icosphere: returns (verts (V,3), faces (F,3)) with outward winding."""
    t = (1.0 + 5 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.asarray(p, np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts), np.array(faces, np.int64)


def mesh_to_tris(verts, faces):
    return np.concatenate([verts[faces[:, 0]], verts[faces[:, 1]], verts[faces[:, 2]]], axis=1)


def box_tris(lo, hi, n=1, inward=False):
    """Closed axis-aligned box as 6 faces, each an n x n grid of quads (2 tris per quad).

    Outward-facing unless inward=True.
    """
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    tris = []
    for axis in range(3):
        for side in (0, 1):
            a1, a2 = (axis + 1) % 3, (axis + 2) % 3
            for i in range(n):
                for j in range(n):
                    def pt(s, t):
                        p = np.empty(3)
                        p[axis] = hi[axis] if side else lo[axis]
                        p[a1] = lo[a1] + (hi[a1] - lo[a1]) * s
                        p[a2] = lo[a2] + (hi[a2] - lo[a2]) * t
                        return p
                    s0, s1, t0, t1 = i / n, (i + 1) / n, j / n, (j + 1) / n
                    q = [pt(s0, t0), pt(s1, t0), pt(s1, t1), pt(s0, t1)]
                    # (a1, a2, axis) is right-handed: counter-clockwise in (a1, a2) faces +axis
                    outward_ccw = (side == 1)
                    if outward_ccw == inward:
                        q = q[::-1]
                    tris.append(np.concatenate([q[0], q[1], q[2]]))
                    tris.append(np.concatenate([q[0], q[2], q[3]]))
    return np.array(tris)


def lens_tris(aperture, radius, nx=64, ny=32):
    """Biconvex lens from two spherical caps (radius `radius`, rim radius `aperture`).

    Each cap is a concentric (Shirley-Chiu) mapping of an nx x ny grid onto the
    rim disk, lifted onto the sphere: 2*nx*ny triangles per cap, less the few chord
    triangles that fall flat in the rim plane at the square's corners. The rim plane is
    z = 0; the caps bulge to +z and -z; both share the rim vertices exactly, so
    the mesh is closed. Normals point outward.
    """
    def disk(a, b):
        if a == 0 and b == 0:
            return 0.0, 0.0
        if abs(a) > abs(b):
            r, phi = a, (math.pi / 4) * (b / a)
        else:
            r, phi = b, math.pi / 2 - (math.pi / 4) * (a / b)
        return r * math.cos(phi), r * math.sin(phi)

    zc = math.sqrt(radius * radius - aperture * aperture)
    grid = np.empty((nx + 1, ny + 1, 3))
    for i in range(nx + 1):
        for j in range(ny + 1):
            x, y = disk(-1 + 2 * i / nx, -1 + 2 * j / ny)
            x, y = x * aperture, y * aperture
            rho2 = min(x * x + y * y, aperture * aperture)
            grid[i, j] = (x, y, math.sqrt(radius * radius - rho2) - zc)
    tris = []
    for sign in (1.0, -1.0):
        g = grid.copy()
        g[..., 2] *= sign
        for i in range(nx):
            for j in range(ny):
                a, b, c, d = g[i, j], g[i + 1, j], g[i + 1, j + 1], g[i, j + 1]
                for tri in ((a, b, c), (a, c, d)):
                    if all(abs(p[2]) < 1e-12 for p in tri):
                        continue    # chord triangle in the rim plane: both caps drop it, the mesh stays closed
                    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
                    if np.dot(n, np.array([0, 0, sign])) < 0:
                        tri = (tri[0], tri[2], tri[1])
                    tris.append(np.concatenate(tri))
    return np.array(tris)


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------

def cornell_glass(width=64, height=64):
    """Five-quad box (open toward the camera) with a glass icosphere and a ceiling light.

    Interior [-.5,.5] x [0,1] x [-.5,.5]; grey albedo 0.7, red/green side walls 0.6;
    icosphere (subdivision 3, 1,280 tris) of radius 0.3 at (0.15, 0.3, -0.1), IOR 1.5;
    a 0.25 x 0.25 light at y = 0.999 facing down with Le = 10; pinhole at (0, .5, 1.8).
    """
    b = Builder()
    grey = b.add_material(material(MAT_LAMBERT, (0.7, 0.7, 0.7)))
    red = b.add_material(material(MAT_LAMBERT, (0.6, 0.0, 0.0)))
    green = b.add_material(material(MAT_LAMBERT, (0.0, 0.6, 0.0)))
    glass = b.add_material(material(MAT_DIELECTRIC, ior=1.5))
    light = b.add_material(material(MAT_LAMBERT, (0.0, 0.0, 0.0), le=(10.0, 10.0, 10.0)))
    x0, x1, y0, y1, z0, z1 = -0.5, 0.5, 0.0, 1.0, -0.5, 0.5
    b.add_quad((x0, y0, z1), (x1, y0, z1), (x1, y0, z0), (x0, y0, z0), grey)     # floor, +y
    b.add_quad((x0, y1, z0), (x1, y1, z0), (x1, y1, z1), (x0, y1, z1), grey)     # ceiling, -y
    b.add_quad((x0, y0, z0), (x1, y0, z0), (x1, y1, z0), (x0, y1, z0), grey)     # back, +z
    b.add_quad((x0, y0, z1), (x0, y0, z0), (x0, y1, z0), (x0, y1, z1), red)      # left, +x
    b.add_quad((x1, y0, z0), (x1, y0, z1), (x1, y1, z1), (x1, y1, z0), green)    # right, -x
    v, f = icosphere(3)
    b.add_tris(mesh_to_tris(v * 0.3 + np.array([0.15, 0.3, -0.1]), f), glass)
    b.add_rect((0.0, 0.999, 0.0), (0.125, 0, 0), (0, 0, 0.125), (0, -1, 0), light, with_uv=True)
    cam = [0.0, 0.5, 1.8, 0.0, 0.5, 0.0, 0.0, 1.0, 0.0, 40.0]
    return b.build(cam, width, height)


def projector(width=512, height=512, key=1):
    """Projector-like caustic: a textured cosine emitter, a biconvex glass lens, a closed room.

    Room [-1,1] x [-1,1] x [-1,1.6] (12 tris, wall albedo U[0.3,0.8] each); lens of two
    spherical caps (R = 0.5, rim radius 0.25, 8,192 tris, IOR 1.5) in the z = 0 plane;
    a 0.2 x 0.2 emitter at z = -0.75 facing +z whose Le is multiplied by a 256 x 256
    checker of 0/1 cells drawn with probability 1/2. Thin-lens focal length about 0.5, so
    the emitter (0.75 behind) is imaged near z = 1.5, at the back wall.
    """
    rng = _rng(key)
    b = Builder()
    lo, hi = np.array([-1.0, -1.0, -1.0]), np.array([1.0, 1.0, 1.6])
    walls = box_tris(lo, hi, n=1, inward=True)
    for k in range(6):
        m = b.add_material(material(MAT_LAMBERT, tuple(rng.uniform(0.3, 0.8, 3))))
        b.add_tris(walls[2 * k: 2 * k + 2], m)
    glass = b.add_material(material(MAT_DIELECTRIC, ior=1.5))
    b.add_tris(lens_tris(0.25, 0.5), glass)
    light = b.add_material(material(MAT_LAMBERT, (0.0, 0.0, 0.0), le=(60.0, 60.0, 60.0), textured=1))
    b.add_rect((0.0, 0.0, -0.75), (0.1, 0, 0), (0, 0.1, 0), (0, 0, 1), light, with_uv=True)
    tex = (rng.uniform(size=(256, 256)) < 0.5).astype(np.float32)
    cam = [0.55, 0.45, -0.95, 0.0, 0.0, 1.6, 0.0, 1.0, 0.0, 55.0]
    return b.build(cam, width, height, tex)


def glossy_procedural(width=1024, height=1024, key=2, target_tris=200_000):
    """Glossy/specular procedural scene of about `target_tris` triangles.

    A room shell with four ceiling quad lights and about 40 objects on a jittered
    grid: displaced icospheres and subdivided boxes, sizes U[0.5, 2] x 0.35.
    Per object: 40 % GGX conductor (roughness U[0.005, 0.1]), 30 % smooth dielectric
    (IOR U[1.3, 1.7]), 30 % Lambert (albedo U[0.2, 0.8]).
    """
    rng = _rng(key)
    b = Builder()
    lo, hi = np.array([-4.0, 0.0, -4.0]), np.array([4.0, 4.0, 4.0])
    shell = b.add_material(material(MAT_LAMBERT, (0.6, 0.6, 0.6)))
    b.add_tris(box_tris(lo, hi, n=1, inward=True), shell)
    lm = b.add_material(material(MAT_LAMBERT, (0.0, 0.0, 0.0), le=(12.0, 12.0, 12.0)))
    for cx, cz in ((-2, -2), (2, -2), (-2, 2), (2, 2)):
        b.add_rect((cx, 3.99, cz), (0.35, 0, 0), (0, 0, 0.35), (0, -1, 0), lm)
    n_obj = 40
    per_obj = (target_tris - 20) / n_obj
    gx, gz = 8, 5
    cells = [(i, j) for i in range(gx) for j in range(gz)]
    for k in range(n_obj):
        i, j = cells[k]
        size = rng.uniform(0.5, 2.0) * 0.35
        cx = -3.5 + 7.0 * (i + 0.5) / gx + rng.uniform(-0.1, 0.1)
        cz = -3.5 + 7.0 * (j + 0.5) / gz + rng.uniform(-0.1, 0.1)
        cy = size + rng.uniform(0.0, 1.5)
        u = rng.uniform()
        if u < 0.4:
            m = b.add_material(material(MAT_CONDUCTOR, tuple(rng.uniform(0.5, 1.0, 3)), roughness=rng.uniform(0.005, 0.1)))
        elif u < 0.7:
            m = b.add_material(material(MAT_DIELECTRIC, ior=rng.uniform(1.3, 1.7)))
        else:
            m = b.add_material(material(MAT_LAMBERT, tuple(rng.uniform(0.2, 0.8, 3))))
        if rng.uniform() < 0.5:
            # displaced icosphere: subdivision chosen to approach the per-object budget
            sub = 4 if per_obj < 12000 else 5
            v, f = icosphere(sub)
            freq = rng.uniform(2.0, 5.0, 3)
            phase = rng.uniform(0, 2 * np.pi, 3)
            disp = 1.0 + 0.12 * np.sin(freq[0] * v[:, 0] + phase[0]) * np.sin(freq[1] * v[:, 1] + phase[1]) \
                * np.sin(freq[2] * v[:, 2] + phase[2])
            v = v * disp[:, None] * size + np.array([cx, cy, cz])
            b.add_tris(mesh_to_tris(v, f), m)
        else:
            n = max(1, int(round(math.sqrt(per_obj / 12.0))))
            ext = size * rng.uniform(0.6, 1.0, 3)
            b.add_tris(box_tris([cx, cy, cz] - ext, [cx, cy, cz] + ext, n=n), m)
    cam = [0.0, 2.2, 3.9, 0.0, 1.0, -1.0, 0.0, 1.0, 0.0, 60.0]
    return b.build(cam, width, height)


def furnace(albedo=0.5, le=1.0, glass_sphere=False, width=16, height=16, sphere_subdiv=2, enclosure="box"):
    """Closed enclosure whose walls all emit Le and reflect with Lambert albedo `albedo`.

    enclosure="box": the 12-triangle cube [-1,1]^3; "sphere": an inward-facing icosphere
    of radius 1.8 (subdivision 3), which has no corners. The camera sits inside. With
    unlimited depth every pixel reads Le / (1 - albedo); with at most K path segments it
    reads Le (1 - albedo^K) / (1 - albedo). glass_sphere=True adds a lossless glass sphere
    (IOR 1.5), which leaves the uniform radiance seen by the camera unchanged.
    """
    b = Builder()
    wall = b.add_material(material(MAT_LAMBERT, (albedo,) * 3, le=(le,) * 3))
    if enclosure == "box":
        b.add_tris(box_tris([-1, -1, -1], [1, 1, 1], n=1, inward=True), wall)
    else:
        v, f = icosphere(3)
        b.add_tris(mesh_to_tris(v * 1.8, f[:, ::-1]), wall)
    if glass_sphere:
        glass = b.add_material(material(MAT_DIELECTRIC, ior=1.5))
        v, f = icosphere(sphere_subdiv)
        b.add_tris(mesh_to_tris(v * 0.45 + np.array([0.1, -0.2, -0.3]), f), glass)
    cam = [0.0, 0.3, 0.9, 0.0, -0.2, -0.3, 0.0, 1.0, 0.0, 70.0]
    return b.build(cam, width, height)


def formfactor_plane(mirror=False, width=8, height=8):
    """A rectangular emitter above a glossy plane (and optionally a mirror).

    mirror=False: emitter [-.5,.5] x [-.25,.25] at y = 1 facing -y, a conductor floor at
    y = 0 (roughness 0.01). The class A, u = 1 incomplete-path density at a floor point is
    the emitter's form factor to that point divided by the emitter area.
    mirror=True: the emitter faces +y at y = 0.5 below a perfect (roughness 0, F0 = 1)
    mirror plane at y = 1.5; a second conductor plane at y = 0 receives L S S paths, whose
    density equals the form factor of the emitter mirrored about y = 1.5 (image method).
    """
    b = Builder()
    floor = b.add_material(material(MAT_CONDUCTOR, (1.0, 1.0, 1.0), roughness=0.01))
    light = b.add_material(material(MAT_LAMBERT, (0.0, 0.0, 0.0), le=(1.0, 1.0, 1.0)))
    b.add_rect((0, 0, 0), (3, 0, 0), (0, 0, 3), (0, 1, 0), floor)
    if not mirror:
        b.add_rect((0, 1.0, 0), (0.5, 0, 0), (0, 0, 0.25), (0, -1, 0), light)
    else:
        mir = b.add_material(material(MAT_CONDUCTOR, (1.0, 1.0, 1.0), roughness=0.0))
        b.add_rect((0, 0.5, 0), (0.5, 0, 0), (0, 0, 0.25), (0, 1, 0), light)
        b.add_rect((0, 1.5, 0), (6, 0, 0), (0, 0, 6), (0, -1, 0), mir)
    cam = [0.0, 2.0, 3.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 40.0]
    return b.build(cam, width, height)


def mirror_room(width=16, height=16, mirror_roughness=0.0):
    """Small diffuse room with a ceiling light, a tilted perfect mirror and a coarse glass ball
    (mirror_roughness > 0: a glossy GGX conductor in place of the perfect mirror).

    Produces short proxy-class paths of both classes (light -> mirror -> floor, light -> glass
    -> floor, light -> wall -> mirror -> floor) that unidirectional path tracing also finds
    at a moderate rate, so the two estimators can be compared pixel by pixel.
    """
    b = Builder()
    wall = b.add_material(material(MAT_LAMBERT, (0.6, 0.6, 0.6)))
    b.add_tris(box_tris([-1, 0, -1], [1, 2, 1], n=1, inward=True), wall)
    light = b.add_material(material(MAT_LAMBERT, (0.0, 0.0, 0.0), le=(8.0, 8.0, 8.0)))
    b.add_rect((0.3, 1.99, 0.0), (0.3, 0, 0), (0, 0, 0.3), (0, -1, 0), light)
    mir = b.add_material(material(MAT_CONDUCTOR, (0.95, 0.95, 0.95), roughness=mirror_roughness))
    c = np.array([-0.6, 1.0, 0.0])
    n = np.array([1.0, -0.35, 0.0])
    n /= np.linalg.norm(n)
    a = np.cross(n, [0.0, 0.0, 1.0])
    a /= np.linalg.norm(a)
    b.add_rect(c, a * 0.45, np.array([0, 0, 0.45]), n, mir)
    glass = b.add_material(material(MAT_DIELECTRIC, ior=1.5))
    v, f = icosphere(1)
    b.add_tris(mesh_to_tris(v * 0.3 + np.array([0.45, 0.6, 0.3]), f), glass)
    cam = [0.0, 1.2, 0.95, 0.0, 0.2, -0.4, 0.0, 1.0, 0.0, 75.0]
    return b.build(cam, width, height)


def serving_scene(seed, width, height, target_tris):
    """One scene of the batched serving workload: a room shell with two ceiling lights and about
    24 objects on a grid, `target_tris` triangles in all. Per object: 25 % perfect mirror, 25 %
    smooth dielectric (IOR U[1.3, 1.7]), 25 % GGX conductor (roughness U[0.001, 0.05]), 25 %
    Lambert (albedo U[0.2, 0.8]); so that mirror/glass chains of several specular vertices occur."""
    rng = _rng(1000 + seed)
    b = Builder()
    lo, hi = np.array([-4.0, 0.0, -4.0]), np.array([4.0, 4.0, 4.0])
    shell = b.add_material(material(MAT_LAMBERT, (0.6, 0.6, 0.6)))
    b.add_tris(box_tris(lo, hi, n=1, inward=True), shell)
    lm = b.add_material(material(MAT_LAMBERT, (0.0, 0.0, 0.0), le=(16.0, 16.0, 16.0)))
    for cx in (-1.5, 1.5):
        b.add_rect((cx, 3.99, 0.0), (0.4, 0, 0), (0, 0, 0.4), (0, -1, 0), lm)
    n_obj = 24
    per_obj = max(20.0, (target_tris - 16) / n_obj)
    gx, gz = 6, 4
    for k in range(n_obj):
        i, j = k % gx, k // gx
        size = rng.uniform(0.5, 2.0) * 0.4
        cx = -3.3 + 6.6 * (i + 0.5) / gx + rng.uniform(-0.1, 0.1)
        cz = -3.3 + 6.6 * (j + 0.5) / gz + rng.uniform(-0.1, 0.1)
        cy = size + rng.uniform(0.0, 1.2)
        u = rng.uniform()
        if u < 0.25:
            m = b.add_material(material(MAT_CONDUCTOR, (0.95, 0.95, 0.95), roughness=0.0))
        elif u < 0.5:
            m = b.add_material(material(MAT_DIELECTRIC, ior=rng.uniform(1.3, 1.7)))
        elif u < 0.75:
            m = b.add_material(material(MAT_CONDUCTOR, tuple(rng.uniform(0.5, 1.0, 3)),
                                        roughness=rng.uniform(0.001, 0.05)))
        else:
            m = b.add_material(material(MAT_LAMBERT, tuple(rng.uniform(0.2, 0.8, 3))))
        if rng.uniform() < 0.5:
            # icosphere with the subdivision closest to the per-object budget (20 * 4^s triangles)
            sub = int(np.clip(round(math.log(per_obj / 20.0, 4)), 0, 8))
            v, f = icosphere(sub)
            freq = rng.uniform(2.0, 5.0, 3)
            phase = rng.uniform(0, 2 * np.pi, 3)
            disp = 1.0 + 0.1 * np.sin(freq[0] * v[:, 0] + phase[0]) * np.sin(freq[1] * v[:, 1] + phase[1]) \
                * np.sin(freq[2] * v[:, 2] + phase[2])
            v = v * disp[:, None] * size + np.array([cx, cy, cz])
            b.add_tris(mesh_to_tris(v, f), m)
        else:
            n = max(1, int(round(math.sqrt(per_obj / 12.0))))
            ext = size * rng.uniform(0.6, 1.0, 3)
            b.add_tris(box_tris([cx, cy, cz] - ext, [cx, cy, cz] + ext, n=n), m)
    cam = [0.0, 2.0, 3.9, 0.0, 1.0, -1.0, 0.0, 1.0, 0.0, 60.0]
    return b.build(cam, width, height)


SERVING_RES = ((256, 256), (640, 480), (1280, 720), (1920, 1080))


def serving_batch(n_scenes=16, key=4, max_tris=2_000_000, res_cap=None):
    """The 16 scenes of the batched serving workload (config 4): scene i has a triangle budget
    drawn log-uniformly from [10^3, max_tris] and a resolution drawn from SERVING_RES (res_cap
    limits the resolution index, for small test runs). Returns a list of (scene, spec) pairs."""
    rng = _rng(key)
    out = []
    for i in range(n_scenes):
        tris = int(round(math.exp(rng.uniform(math.log(1e3), math.log(max_tris)))))
        r = int(rng.integers(0, len(SERVING_RES)))
        if res_cap is not None:
            r = min(r, res_cap)
        w, h = SERVING_RES[r]
        sc = serving_scene(i, w, h, tris)
        out.append((sc, dict(target_tris=tris, width=w, height=h)))
    return out


CONFIGS = {
    0: dict(scene=lambda: cornell_glass(64, 64), spp=16, max_depth=8, n_light=4096, cand_cap=400,
            n_subspaces=64, n_spec=64, n_ctrl=10, seed=0),
    1: dict(scene=lambda: projector(512, 512), spp=64, max_depth=12, n_light=500_000, cand_cap=20_000,
            n_subspaces=1000, n_spec=100, n_ctrl=10, seed=0),
    2: dict(scene=lambda: glossy_procedural(1024, 1024), spp=256, max_depth=12, n_light=262_144,
            cand_cap=10_486, n_subspaces=1000, n_spec=100, n_ctrl=10, seed=0),
    # config 2's scene with the learned selection: 10 % defensive plain sampling, online training
    # on up to 65,536 contribution samples per iteration, Adam step 1e-3
    3: dict(scene=lambda: glossy_procedural(1024, 1024), spp=256, max_depth=12, n_light=262_144,
            cand_cap=10_486, n_subspaces=1000, n_spec=100, n_ctrl=10, seed=0, mlp=True, mlp_mix=0.9,
            mlp_lr=1e-3, train_iters=1_000_000),
}


def config(cfg_id):
    c = dict(CONFIGS[cfg_id])
    c["scene"] = c["scene"]()
    return c


def tri_count(scene):
    return int(scene["tri"].shape[0])


def planes_scene(width=64, height=64, sigma_s=0.5, sigma_t=0.6):
    """The photon-plane workload (single scattering, Section 6.7's volumetric setting): a 1.0 x 0.6
    rectangular Lambertian light 1.5 above the origin facing down (radiance 4), a homogeneous
    medium filling space (isotropic phase function, sigma_s, sigma_t), nothing occluding, and a
    pinhole camera below and in front looking up into the lit column (eye rays 15 to 40 degrees
    above the light's plane, ending at t_max = 3.5, at least ~0.27 from the light). No eye ray runs
    parallel to the light: there the CMIS estimate of a grazing plane grows like 1 / cos(theta)
    and its variance diverges."""
    return {
        "light_c": np.array([0.0, 1.5, 0.0]), "light_u": np.array([1.0, 0.0, 0.0]),
        "light_v": np.array([0.0, 0.0, 1.0]),   # emits toward u x v = (0, -1, 0)
        "light_eu": 0.5, "light_ev": 0.3, "le": np.array([4.0, 4.0, 4.0]),
        "camera": np.array([0.0, -1.0, 2.5, 0.0, 0.3, 0.0, 0.0, 1.0, 0.0, 24.0]),
        "sigma_s": float(sigma_s), "sigma_t": float(sigma_t), "t_max": 3.5,
        "width": int(width), "height": int(height),
    }
