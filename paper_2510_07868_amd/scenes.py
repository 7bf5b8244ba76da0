"""Seeded synthetic scenes: the inputs of the renderer and of its CPU oracle.

This module only builds geometry, materials and cameras as plain arrays.  It holds
none of the rendering arithmetic (no intersection, sampling, roulette or
network code), so that both the HIP path and the oracle can take their inputs
from it without sharing any of the method's code.

The paper's own scenes (apartments, Bistro, Sponza, Sun Temple, Cornell at
1280x720 / 750x750, Sec. 6) are not available; these procedural scenes stand in
for them with the shapes and sizes of the benchmark configurations:

* ``cornell``     36 triangles, grey Lambertian 0.7, one quad light L_e=10.
* ``heightfield`` about 1.05 M triangles: displaced 1024x1024 fBm heightfield
                  meshed at 725x725 vertices + 200 random boxes, 30 % GGX.
* ``room``        about 2.1 M triangles: room whose only light is outside a
                  0.5 m^2 ceiling opening (the paper's "area light positioned
                  outside" case), 1024x1024-vertex floor heightfield + 200 boxes.
* ``terrain5m``   about 5.0 M triangles: 1581x1581-vertex heightfield + 2000
                  boxes (flattened), 30 % GGX; ``terrain5m_instanced`` the same
                  scene with the boxes as 2000 instances of one unit box.
* ``cornell_instanced`` the Cornell box with its two boxes as instances;
  ``instance_field`` 64 instances of two meshes under random rotations,
                  non-uniform scales and one mirror, over a floor.
* ``furnace``     closed grey box (rho 0.7, L_e 1 everywhere): closed-form image.
* ``two_triangle`` a 2x2-pixel scene small enough for exhaustive enumeration.

Materials are rows ``(rho_r, rho_g, rho_b, alpha, Le_r, Le_g, Le_b)`` with a type
code; ``rho`` is the Lambertian albedo or the GGX F0.  Cameras are
``(eye xyz, look-at xyz, up xyz, vertical fov in degrees)``.  Triangles are
wound so that ``cross(v1-v0, v2-v0)`` points to the emitting (front) side.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

MAT_LAMBERT = 0
MAT_GGX = 1
MAT_EMITTER = 2


NO_MATERIAL = 0xFFFFFFFF  # an instance that keeps its mesh's own materials


@dataclasses.dataclass
class Scene:
    name: str
    verts: np.ndarray      # float32 [nv, 3]
    tris: np.ndarray       # uint32  [nt, 3]
    tri_mat: np.ndarray    # uint32  [nt]
    mat_type: np.ndarray   # uint32  [nm]
    mat_params: np.ndarray  # float32 [nm, 7]
    camera: np.ndarray     # float32 [10]
    env: np.ndarray        # float32 [3]

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])


@dataclasses.dataclass
class InstancedScene:
    """A world-space base mesh plus instances of object-space meshes.

    ``base`` holds the base triangles (possibly none), all materials, the camera and the
    environment.  Mesh m is triangles ``mesh_tri_begin[m] .. mesh_tri_begin[m+1]`` of
    ``mesh_tris`` / ``mesh_tri_mat`` over ``mesh_verts``.  Instance j places mesh
    ``inst_mesh[j]`` by the row-major 3x4 object-to-world map ``inst_xform[j]`` (world = A x + t)
    with material ``inst_mat[j]`` for all its triangles, or NO_MATERIAL for the mesh's own."""
    name: str
    base: Scene
    mesh_verts: np.ndarray      # float32 [nv, 3]
    mesh_tris: np.ndarray       # uint32  [nt, 3]
    mesh_tri_mat: np.ndarray    # uint32  [nt]
    mesh_tri_begin: np.ndarray  # uint64  [n_meshes + 1]
    inst_mesh: np.ndarray       # uint32  [ni]
    inst_xform: np.ndarray      # float32 [ni, 12]
    inst_mat: np.ndarray        # uint32  [ni]

    @property
    def n_tris(self) -> int:
        """Triangles after flattening."""
        sizes = np.diff(self.mesh_tri_begin.astype(np.int64))
        return int(self.base.tris.shape[0] + sizes[self.inst_mesh].sum())

    @property
    def workspace_tris(self) -> int:
        """Triangle slots the renderer's workspace needs: base and mesh triangles, 3 per
        instance record (the base mesh is one)."""
        return int(self.base.tris.shape[0] + self.mesh_tris.shape[0] + 3 * (self.inst_mesh.shape[0] + 1))

    def flatten(self) -> Scene:
        """The same scene as one world-space triangle list: the base triangles, then every
        instance's mesh triangles in mesh order at world positions ((a00 x + a01 y) + a02 z) + t0
        (and likewise for y, z), evaluated in float64 and rounded to float32."""
        verts = [self.base.verts.astype(np.float32).reshape(-1, 3)]
        tris = [self.base.tris.astype(np.int64).reshape(-1, 3)]
        mats = [self.base.tri_mat.astype(np.int64)]
        nv = verts[0].shape[0]
        beg = self.mesh_tri_begin.astype(np.int64)
        mv = self.mesh_verts.astype(np.float64)
        for j in range(self.inst_mesh.shape[0]):
            m = int(self.inst_mesh[j])
            mt = self.mesh_tris[beg[m]:beg[m + 1]].astype(np.int64)
            p = mv[mt.reshape(-1)]  # corners, 3 per triangle
            x = self.inst_xform[j].astype(np.float64).reshape(3, 4)
            w = np.empty_like(p)
            for a in range(3):
                w[:, a] = ((x[a, 0] * p[:, 0] + x[a, 1] * p[:, 1]) + x[a, 2] * p[:, 2]) + x[a, 3]
            verts.append(w.astype(np.float32))
            tris.append(nv + np.arange(3 * mt.shape[0], dtype=np.int64).reshape(-1, 3))
            nv += w.shape[0]
            if int(self.inst_mat[j]) == NO_MATERIAL:
                mats.append(self.mesh_tri_mat[beg[m]:beg[m + 1]].astype(np.int64))
            else:
                mats.append(np.full(mt.shape[0], int(self.inst_mat[j]), np.int64))
        b = self.base
        return Scene(name=self.name + "_flat", verts=np.ascontiguousarray(np.concatenate(verts).astype(np.float32)),
                     tris=np.ascontiguousarray(np.concatenate(tris).astype(np.uint32)),
                     tri_mat=np.ascontiguousarray(np.concatenate(mats).astype(np.uint32)),
                     mat_type=b.mat_type.copy(), mat_params=b.mat_params.copy(), camera=b.camera.copy(),
                     env=b.env.copy())


_BOX_FACES = [  # (corner ids in cyclic order, outward local normal)
    ([0, 1, 3, 2], (-1, 0, 0)), ([4, 6, 7, 5], (1, 0, 0)),
    ([0, 4, 5, 1], (0, -1, 0)), ([2, 3, 7, 6], (0, 1, 0)),
    ([0, 2, 6, 4], (0, 0, -1)), ([1, 5, 7, 3], (0, 0, 1)),
]


def _yaw_box_xform(center, size, yaw) -> np.ndarray:
    """Object-to-world map of the unit box to an axis box of ``size`` rotated by ``yaw`` about
    +y at ``center`` (row-major 3x4)."""
    cy, sy_ = math.cos(yaw), math.sin(yaw)
    rot = np.array([[cy, 0.0, sy_], [0.0, 1.0, 0.0], [-sy_, 0.0, cy]])
    a = rot * np.asarray(size, np.float64)[None, :]
    return np.concatenate([a, np.asarray(center, np.float64).reshape(3, 1)], axis=1).reshape(12)


class _Builder:
    def __init__(self):
        self.v = []
        self.t = []
        self.m = []
        self.nv = 0
        self.mat_type = []
        self.mat_params = []
        # object-space meshes and their instances
        self.ov = []
        self.ot = []
        self.om = []
        self.onv = 0
        self.obeg = [0]
        self.inst = []  # (mesh, xform[12], material)

    def object_mesh(self, verts, tris, mat=NO_MATERIAL) -> int:
        verts = np.asarray(verts, np.float64).reshape(-1, 3)
        tris = np.asarray(tris, np.int64).reshape(-1, 3)
        self.ov.append(verts)
        self.ot.append(tris + self.onv)
        self.om.append(np.full(tris.shape[0], 0 if mat == NO_MATERIAL else mat, np.int64))
        self.onv += verts.shape[0]
        self.obeg.append(self.obeg[-1] + tris.shape[0])
        return len(self.obeg) - 2

    def unit_box_mesh(self) -> int:
        """The axis box [-0.5, 0.5]^3 as an object mesh, 12 triangles facing out."""
        corners = np.array([[x, y, z] for x in (-0.5, 0.5) for y in (-0.5, 0.5) for z in (-0.5, 0.5)])
        vs, ts = [], []
        for ids, nloc in _BOX_FACES:
            p = corners[ids]
            if np.dot(np.cross(p[1] - p[0], p[2] - p[0]), nloc) < 0:
                p = p[::-1].copy()
            base = sum(len(q) for q in vs)
            vs.append(p)
            ts.append(np.array([[0, 1, 2], [0, 2, 3]]) + base)
        return self.object_mesh(np.concatenate(vs), np.concatenate(ts))

    def instance(self, mesh, xform, mat=NO_MATERIAL):
        self.inst.append((int(mesh), np.asarray(xform, np.float64).reshape(12), int(mat)))

    def material(self, mtype, rho, alpha=1.0, le=(0.0, 0.0, 0.0)) -> int:
        self.mat_type.append(int(mtype))
        rho = np.broadcast_to(np.asarray(rho, np.float64), (3,))
        le = np.broadcast_to(np.asarray(le, np.float64), (3,))
        self.mat_params.append([rho[0], rho[1], rho[2], alpha, le[0], le[1], le[2]])
        return len(self.mat_type) - 1

    def mesh(self, verts, tris, mat):
        verts = np.asarray(verts, np.float64).reshape(-1, 3)
        tris = np.asarray(tris, np.int64).reshape(-1, 3)
        self.v.append(verts)
        self.t.append(tris + self.nv)
        self.m.append(np.full(tris.shape[0], mat, np.int64))
        self.nv += verts.shape[0]

    def quad(self, center, u, v, normal, mat):
        """Rectangle center +- u/2 +- v/2 whose front side faces ``normal``."""
        c, u, v = (np.asarray(a, np.float64) for a in (center, u, v))
        p = np.array([c - u / 2 - v / 2, c + u / 2 - v / 2, c + u / 2 + v / 2, c - u / 2 + v / 2])
        if np.dot(np.cross(p[1] - p[0], p[2] - p[0]), normal) < 0:
            p = p[::-1].copy()
        self.mesh(p, [[0, 1, 2], [0, 2, 3]], mat)

    def box(self, center, size, yaw, mat, inward=False):
        """Axis box rotated by ``yaw`` about +y; 12 triangles facing out (or in)."""
        c = np.asarray(center, np.float64)
        sx, sy, sz = (float(s) for s in size)
        cy, sy_ = math.cos(yaw), math.sin(yaw)
        rot = np.array([[cy, 0.0, sy_], [0.0, 1.0, 0.0], [-sy_, 0.0, cy]])
        corners = np.array([[x, y, z] for x in (-0.5, 0.5) for y in (-0.5, 0.5) for z in (-0.5, 0.5)])
        corners = corners * np.array([sx, sy, sz])
        pts = corners @ rot.T + c
        faces = [  # (corner ids in cyclic order, outward local normal)
            ([0, 1, 3, 2], (-1, 0, 0)), ([4, 6, 7, 5], (1, 0, 0)),
            ([0, 4, 5, 1], (0, -1, 0)), ([2, 3, 7, 6], (0, 1, 0)),
            ([0, 2, 6, 4], (0, 0, -1)), ([1, 5, 7, 3], (0, 0, 1)),
        ]
        for ids, nloc in faces:
            n = rot @ np.asarray(nloc, np.float64)
            if inward:
                n = -n
            p = pts[ids]
            if np.dot(np.cross(p[1] - p[0], p[2] - p[0]), n) < 0:
                p = p[::-1].copy()
            self.mesh(p, [[0, 1, 2], [0, 2, 3]], mat)

    def build(self, name, camera, env) -> Scene:
        verts = np.concatenate(self.v).astype(np.float32) if self.v else np.zeros((0, 3), np.float32)
        tris = np.concatenate(self.t).astype(np.uint32) if self.t else np.zeros((0, 3), np.uint32)
        tri_mat = np.concatenate(self.m).astype(np.uint32) if self.m else np.zeros(0, np.uint32)
        return Scene(
            name=name,
            verts=np.ascontiguousarray(verts),
            tris=np.ascontiguousarray(tris),
            tri_mat=np.ascontiguousarray(tri_mat),
            mat_type=np.asarray(self.mat_type, np.uint32),
            mat_params=np.asarray(self.mat_params, np.float32).reshape(-1, 7),
            camera=np.asarray(camera, np.float32).reshape(10),
            env=np.broadcast_to(np.asarray(env, np.float32), (3,)).copy(),
        )


    def build_instanced(self, name, camera, env) -> InstancedScene:
        base = self.build(name, camera, env)
        return InstancedScene(
            name=name, base=base,
            mesh_verts=np.ascontiguousarray(np.concatenate(self.ov).astype(np.float32)),
            mesh_tris=np.ascontiguousarray(np.concatenate(self.ot).astype(np.uint32)),
            mesh_tri_mat=np.ascontiguousarray(np.concatenate(self.om).astype(np.uint32)),
            mesh_tri_begin=np.asarray(self.obeg, np.uint64),
            inst_mesh=np.asarray([i[0] for i in self.inst], np.uint32),
            inst_xform=np.ascontiguousarray(np.stack([i[1] for i in self.inst]).astype(np.float32)),
            inst_mat=np.asarray([i[2] for i in self.inst], np.uint32),
        )


def _cornell_boxes(b: _Builder, mat):
    b.box((0.66, 0.15, 0.35), (0.3, 0.3, 0.3), math.radians(-18.0), mat)
    b.box((0.33, 0.30, 0.65), (0.3, 0.6, 0.3), math.radians(17.0), mat)


def cornell() -> Scene:
    """Cornell box in [0,1]^3 open towards -z: 5 walls + 2 boxes = 34 triangles, 1 quad light."""
    b = _Builder()
    grey = b.material(MAT_LAMBERT, 0.7)
    light = b.material(MAT_EMITTER, 0.0, 1.0, 10.0)
    b.quad((0.5, 0.0, 0.5), (1, 0, 0), (0, 0, 1), (0, 1, 0), grey)    # floor
    b.quad((0.5, 1.0, 0.5), (1, 0, 0), (0, 0, 1), (0, -1, 0), grey)   # ceiling
    b.quad((0.5, 0.5, 1.0), (1, 0, 0), (0, 1, 0), (0, 0, -1), grey)   # back
    b.quad((0.0, 0.5, 0.5), (0, 1, 0), (0, 0, 1), (1, 0, 0), grey)    # left
    b.quad((1.0, 0.5, 0.5), (0, 1, 0), (0, 0, 1), (-1, 0, 0), grey)   # right
    _cornell_boxes(b, grey)
    b.quad((0.5, 0.999, 0.5), (0.25, 0, 0), (0, 0, 0.25), (0, -1, 0), light)
    cam = (0.5, 0.5, -1.4, 0.5, 0.5, 0.5, 0.0, 1.0, 0.0, 40.0)
    return b.build("cornell", cam, 0.0)


def cornell_instanced() -> InstancedScene:
    """The Cornell box with its two boxes as instances of one unit box (36 triangles flattened)."""
    b = _Builder()
    grey = b.material(MAT_LAMBERT, 0.7)
    light = b.material(MAT_EMITTER, 0.0, 1.0, 10.0)
    b.quad((0.5, 0.0, 0.5), (1, 0, 0), (0, 0, 1), (0, 1, 0), grey)    # floor
    b.quad((0.5, 1.0, 0.5), (1, 0, 0), (0, 0, 1), (0, -1, 0), grey)   # ceiling
    b.quad((0.5, 0.5, 1.0), (1, 0, 0), (0, 1, 0), (0, 0, -1), grey)   # back
    b.quad((0.0, 0.5, 0.5), (0, 1, 0), (0, 0, 1), (1, 0, 0), grey)    # left
    b.quad((1.0, 0.5, 0.5), (0, 1, 0), (0, 0, 1), (-1, 0, 0), grey)   # right
    b.quad((0.5, 0.999, 0.5), (0.25, 0, 0), (0, 0, 0.25), (0, -1, 0), light)
    box = b.unit_box_mesh()
    b.instance(box, _yaw_box_xform((0.66, 0.15, 0.35), (0.3, 0.3, 0.3), math.radians(-18.0)), grey)
    b.instance(box, _yaw_box_xform((0.33, 0.30, 0.65), (0.3, 0.6, 0.3), math.radians(17.0)), grey)
    cam = (0.5, 0.5, -1.4, 0.5, 0.5, 0.5, 0.0, 1.0, 0.0, 40.0)
    return b.build_instanced("cornell_instanced", cam, 0.0)


def instance_field(seed: int = 0, n: int = 64) -> InstancedScene:
    """A 4x4 m floor with two quad lights above and ``n`` instances of two meshes (a unit box
    and an irregular tetrahedron with its own GGX material) under random 3D rotations and
    non-uniform scales; instance 0 is mirrored (det < 0)."""
    rng = np.random.default_rng(seed)
    b = _Builder()
    floor = b.material(MAT_LAMBERT, 0.6)
    light = b.material(MAT_EMITTER, 0.0, 1.0, 15.0)
    b.quad((2.0, 0.0, 2.0), (4, 0, 0), (0, 0, 4), (0, 1, 0), floor)
    b.quad((1.0, 3.0, 1.5), (0.8, 0, 0), (0, 0, 0.8), (0, -1, 0), light)
    b.quad((3.0, 3.0, 2.5), (0.8, 0, 0), (0, 0, 0.8), (0, -1, 0), light)
    box = b.unit_box_mesh()
    tet_mat = b.material(MAT_GGX, (0.8, 0.6, 0.3), 0.2)
    tv = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1], [0.3, 0.2, 1.1]]) - 0.4
    tet = b.object_mesh(tv, [[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]], tet_mat)
    mats = [b.material(MAT_LAMBERT, rng.uniform(0.1, 0.9, size=3)) for _ in range(4)]
    for j in range(n):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        rot = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        scale = rng.uniform(0.1, 0.5, size=3)
        if j == 0:
            scale[0] = -scale[0]
        a = rot * scale[None, :]
        c = np.array([rng.uniform(0.3, 3.7), rng.uniform(0.2, 1.5), rng.uniform(0.3, 3.7)])
        xf = np.concatenate([a, c.reshape(3, 1)], axis=1).reshape(12)
        if j % 3 == 2:
            b.instance(tet, xf)
        else:
            b.instance(box, xf, mats[j % 4])
    cam = (2.0, 1.8, -2.5, 2.0, 0.6, 2.0, 0.0, 1.0, 0.0, 55.0)
    return b.build_instanced("instance_field", cam, 0.05)


def instances_only(seed: int = 0) -> InstancedScene:
    """No base mesh: a floor (a flattened unit box), 24 boxes and two emitting quads, all
    instances — the quads of one emitting mesh placed twice, so that the light list is made of
    instance triangles."""
    rng = np.random.default_rng(seed)
    b = _Builder()
    grey = b.material(MAT_LAMBERT, 0.6)
    light = b.material(MAT_EMITTER, 0.0, 1.0, 12.0)
    box = b.unit_box_mesh()
    # a unit quad in the xz plane facing -y (down), emitting
    quad = b.object_mesh([[-0.5, 0.0, -0.5], [0.5, 0.0, -0.5], [0.5, 0.0, 0.5], [-0.5, 0.0, 0.5]],
                         [[0, 1, 2], [0, 2, 3]], light)
    b.instance(box, _yaw_box_xform((2.0, -0.05, 2.0), (4.0, 0.1, 4.0), 0.0), grey)
    for _ in range(24):
        sx, sy, sz = rng.uniform(0.1, 0.6, size=3)
        x, z = rng.uniform(0.3, 3.7, size=2)
        m = b.material(MAT_GGX, rng.uniform(0.2, 0.9, size=3), float(rng.uniform(0.1, 0.5))) if rng.uniform() < 0.3 \
            else b.material(MAT_LAMBERT, rng.uniform(0.1, 0.9, size=3))
        b.instance(box, _yaw_box_xform((x, sy / 2, z), (sx, sy, sz), float(rng.uniform(0, 2 * math.pi))), m)
    for c in ((1.2, 2.5, 1.5), (2.8, 2.5, 2.6)):
        b.instance(quad, _yaw_box_xform(c, (0.7, 1.0, 0.7), 0.3))
    cam = (2.0, 1.6, -2.0, 2.0, 0.4, 2.0, 0.0, 1.0, 0.0, 55.0)
    return b.build_instanced("instances_only", cam, 0.02)


def furnace(albedo: float = 0.7, emission: float = 1.0) -> Scene:
    """Closed grey box plus the Cornell boxes; every surface reflects ``albedo`` and emits ``emission``."""
    b = _Builder()
    m = b.material(MAT_LAMBERT, albedo, 1.0, emission)
    b.box((0.5, 0.5, 0.5), (1.0, 1.0, 1.0), 0.0, m, inward=True)
    _cornell_boxes(b, m)
    cam = (0.5, 0.5, 0.05, 0.5, 0.5, 1.0, 0.0, 1.0, 0.0, 60.0)
    return b.build("furnace", cam, 0.0)


def two_triangle() -> Scene:
    """Two triangles seen by a 2x2 camera: a floor reflector R and an emitting back wall E, env 0.25."""
    b = _Builder()
    e = b.material(MAT_LAMBERT, 0.5, 1.0, 4.0)
    r = b.material(MAT_LAMBERT, (0.3, 0.6, 0.2))
    b.mesh([(-6.0, -1.0, -2.0), (0.0, -1.0, 8.0), (6.0, -1.0, -2.0)], [[0, 1, 2]], r)   # floor, faces +y
    b.mesh([(-6.0, -6.0, 3.0), (0.0, 8.0, 3.0), (6.0, -6.0, 3.0)], [[0, 1, 2]], e)     # wall, faces -z
    cam = (0.0, 0.0, -2.0, 0.0, -0.5, 3.0, 0.0, 1.0, 0.0, 60.0)
    return b.build("two_triangle", cam, 0.25)


def _value_noise_fbm(res: int, octaves: int, rng: np.random.Generator, base: int = 8) -> np.ndarray:
    """res x res fBm of smoothstep-interpolated lattice noise, normalised to [-1, 1]."""
    out = np.zeros((res, res), np.float64)
    amp, total = 1.0, 0.0
    x = np.linspace(0.0, 1.0, res, endpoint=False) + 0.5 / res
    for o in range(octaves):
        cells = base << o
        lat = rng.uniform(-1.0, 1.0, size=(cells + 1, cells + 1))
        gx = x * cells
        i0 = np.floor(gx).astype(np.int64)
        f = gx - i0
        s = f * f * (3.0 - 2.0 * f)
        a = lat[i0][:, i0]
        bq = lat[i0][:, i0 + 1]
        c = lat[i0 + 1][:, i0]
        d = lat[i0 + 1][:, i0 + 1]
        sy = s[:, None]
        sx = s[None, :]
        out += amp * ((a * (1 - sx) + bq * sx) * (1 - sy) + (c * (1 - sx) + d * sx) * sy)
        total += amp
        amp *= 0.5
    return out / total


def _sample_bilinear(tex: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    res = tex.shape[0]
    x = np.clip(u * (res - 1), 0, res - 1 - 1e-9)
    y = np.clip(v * (res - 1), 0, res - 1 - 1e-9)
    x0 = np.floor(x).astype(np.int64)
    y0 = np.floor(y).astype(np.int64)
    fx = x - x0
    fy = y - y0
    return (tex[y0, x0] * (1 - fx) * (1 - fy) + tex[y0, x0 + 1] * fx * (1 - fy)
            + tex[y0 + 1, x0] * (1 - fx) * fy + tex[y0 + 1, x0 + 1] * fx * fy)


def _heightfield(b: _Builder, size: float, nvert: int, amplitude: float, offset: float,
                 tex: np.ndarray, mat: int, origin=(0.0, 0.0)):
    """Grid mesh of nvert x nvert vertices over [0,size]^2 displaced by ``tex``; faces +y."""
    g = np.linspace(0.0, 1.0, nvert)
    uu, vv = np.meshgrid(g, g)             # uu along x, vv along z
    h = offset + amplitude * _sample_bilinear(tex, uu, vv)
    verts = np.stack([origin[0] + uu * size, h, origin[1] + vv * size], axis=-1).reshape(-1, 3)
    i = np.arange(nvert - 1)
    ii, jj = np.meshgrid(i, i)             # ii along x, jj along z
    a = (jj * nvert + ii).reshape(-1)
    bb = a + 1
    c = a + nvert
    d = c + 1
    # cross(v1-v0, v2-v0) must point to +y: (a, c, b) and (b, c, d)
    tris = np.concatenate([np.stack([a, c, bb], -1), np.stack([bb, c, d], -1)])
    b.mesh(verts, tris, mat)
    return h


def _random_boxes(b: _Builder, rng, n, extent, height_fn, ggx_frac=0.3, mesh=None):
    """n boxes on the heightfield; with ``mesh`` (a unit box object mesh) as instances of it."""
    for _ in range(n):
        sx, sy, sz = rng.uniform(0.1, 0.8, size=3)
        x, z = rng.uniform(0.0, extent, size=2)
        yaw = rng.uniform(0.0, 2.0 * math.pi)
        base = height_fn(x, z)
        if rng.uniform() < ggx_frac:
            m = b.material(MAT_GGX, rng.uniform(0.1, 0.9, size=3), float(rng.uniform(0.05, 0.5)))
        else:
            m = b.material(MAT_LAMBERT, rng.uniform(0.1, 0.9, size=3))
        if mesh is None:
            b.box((x, base + sy / 2 - 0.05, z), (sx, sy, sz), yaw, m)
        else:
            b.instance(mesh, _yaw_box_xform((x, base + sy / 2 - 0.05, z), (sx, sy, sz), yaw), m)


def heightfield(seed: int = 0) -> Scene:
    """~1.05 M triangles: 725x725-vertex mesh of a 1024x1024 fBm texture over 10x10 m + 200 boxes."""
    rng = np.random.default_rng(seed)
    b = _Builder()
    tex = _value_noise_fbm(1024, 4, rng)
    ground = b.material(MAT_LAMBERT, rng.uniform(0.1, 0.9, size=3))
    _heightfield(b, 10.0, 725, 0.5, 0.0, tex, ground)
    hf = lambda x, z: 0.5 * float(_sample_bilinear(tex, np.array(x / 10.0), np.array(z / 10.0)))
    _random_boxes(b, rng, 200, 10.0, hf)
    light = b.material(MAT_EMITTER, 0.0, 1.0, 20.0)
    b.quad((3.0, 4.0, 3.0), (1, 0, 0), (0, 0, 1), (0, -1, 0), light)
    b.quad((7.0, 4.0, 7.0), (1, 0, 0), (0, 0, 1), (0, -1, 0), light)
    cam = (5.0, 3.0, -2.0, 5.0, 0.0, 5.0, 0.0, 1.0, 0.0, 50.0)
    return b.build("heightfield", cam, 0.1)


def room(seed: int = 0) -> Scene:
    """~2.1 M triangles: 10x4x10 m room lit only through a 0.5 m^2 ceiling opening."""
    rng = np.random.default_rng(seed)
    b = _Builder()
    wall = b.material(MAT_LAMBERT, 0.7)
    tex = _value_noise_fbm(1024, 4, rng)
    floor = b.material(MAT_LAMBERT, rng.uniform(0.1, 0.9, size=3))
    _heightfield(b, 10.0, 1024, 0.25, 0.25, tex, floor)
    hf = lambda x, z: 0.25 + 0.25 * float(_sample_bilinear(tex, np.array(x / 10.0), np.array(z / 10.0)))
    _random_boxes(b, rng, 200, 10.0, hf)
    # walls (inward), y in [0, 4]
    b.quad((5.0, 2.0, 0.0), (10, 0, 0), (0, 4, 0), (0, 0, 1), wall)
    b.quad((5.0, 2.0, 10.0), (10, 0, 0), (0, 4, 0), (0, 0, -1), wall)
    b.quad((0.0, 2.0, 5.0), (0, 0, 10), (0, 4, 0), (1, 0, 0), wall)
    b.quad((10.0, 2.0, 5.0), (0, 0, 10), (0, 4, 0), (-1, 0, 0), wall)
    # ceiling with a square hole of side s centred at (5, 4, 5)
    s = math.sqrt(0.5)
    lo, hi = 5.0 - s / 2, 5.0 + s / 2
    for (x0, x1, z0, z1) in ((0.0, 10.0, 0.0, lo), (0.0, 10.0, hi, 10.0), (0.0, lo, lo, hi), (hi, 10.0, lo, hi)):
        b.quad(((x0 + x1) / 2, 4.0, (z0 + z1) / 2), (x1 - x0, 0, 0), (0, 0, z1 - z0), (0, -1, 0), wall)
    light = b.material(MAT_EMITTER, 0.0, 1.0, 50.0)
    b.quad((5.0, 6.0, 5.0), (2, 0, 0), (0, 0, 2), (0, -1, 0), light)
    cam = (1.0, 2.0, 1.0, 6.0, 0.5, 6.0, 0.0, 1.0, 0.0, 60.0)
    return b.build("room", cam, 0.1)


def _terrain5m(seed: int, instanced: bool):
    rng = np.random.default_rng(seed)
    b = _Builder()
    tex = _value_noise_fbm(1024, 4, rng)
    ground = b.material(MAT_LAMBERT, rng.uniform(0.1, 0.9, size=3))
    _heightfield(b, 20.0, 1581, 0.5, 0.0, tex, ground)
    hf = lambda x, z: 0.5 * float(_sample_bilinear(tex, np.array(x / 20.0), np.array(z / 20.0)))
    _random_boxes(b, rng, 2000, 20.0, hf, mesh=b.unit_box_mesh() if instanced else None)
    light = b.material(MAT_EMITTER, 0.0, 1.0, 20.0)
    b.quad((6.0, 4.0, 6.0), (2, 0, 0), (0, 0, 2), (0, -1, 0), light)
    b.quad((14.0, 4.0, 14.0), (2, 0, 0), (0, 0, 2), (0, -1, 0), light)
    cam = (10.0, 4.0, -3.0, 10.0, 0.0, 10.0, 0.0, 1.0, 0.0, 50.0)
    if instanced:
        return b.build_instanced("terrain5m_instanced", cam, 0.1)
    return b.build("terrain5m", cam, 0.1)


def terrain5m(seed: int = 0) -> Scene:
    """~5.0 M triangles: 1581x1581-vertex heightfield over 20x20 m + 2000 boxes (flattened)."""
    return _terrain5m(seed, False)


def terrain5m_instanced(seed: int = 0) -> InstancedScene:
    """terrain5m with its 2000 boxes as instances of one unit box (same random draws)."""
    return _terrain5m(seed, True)


SCENES = {
    "cornell": cornell,
    "furnace": furnace,
    "two_triangle": two_triangle,
    "heightfield": heightfield,
    "room": room,
    "terrain5m": terrain5m,
    "cornell_instanced": cornell_instanced,
    "instance_field": instance_field,
    "terrain5m_instanced": terrain5m_instanced,
    "instances_only": instances_only,
}

