"""Instanced scenes (a base mesh plus placed copies of object-space meshes): their flattened
form, which the oracle traces, is the same geometry as the scene built without instances, and
placed triangles keep their winding (a mirror reverses their front side)."""
import math

import numpy as np


def _tri_keys(sc):
    v = sc.verts.astype(np.float64)[sc.tris.astype(np.int64)]  # [nt, 3, 3]
    return v, sc.tri_mat.astype(np.int64)


def test_cornell_instanced_flattens_to_the_cornell_box(scenes):
    flat = scenes.cornell_instanced().flatten()
    ref = scenes.cornell()
    assert flat.n_tris == ref.n_tris == 36
    vf, mf = _tri_keys(flat)
    vr, mr = _tri_keys(ref)
    used = np.zeros(flat.n_tris, bool)
    for k in range(ref.n_tris):
        # the same corners in the same cyclic order (winding), within float32 rounding of the map
        match = None
        for j in np.nonzero(~used)[0]:
            for rot in range(3):
                if np.allclose(np.roll(vf[j], rot, axis=0), vr[k], atol=1e-6) and mf[j] == mr[k]:
                    match = j
            if match is not None:
                break
        assert match is not None, k
        used[match] = True
    assert used.all()


def test_instanced_scene_sizes(scenes):
    s = scenes.instance_field(0, 64)
    sizes = np.diff(s.mesh_tri_begin.astype(np.int64))
    assert list(sizes) == [12, 4]
    assert s.n_tris == s.base.n_tris + int(sizes[s.inst_mesh].sum()) == s.flatten().n_tris
    assert s.workspace_tris == s.base.n_tris + 16 + 3 * 65


def test_flattened_instances_keep_their_winding(scenes):
    # a triangle's front side is that of cross(v1 - v0, v2 - v0) of its placed corners: outward
    # for the meshes under proper maps, inward under the mirror (det < 0 reverses the winding;
    # only emitters are one-sided, and the renderer's triangles are the same placed corners)
    s = scenes.instance_field(0, 64)
    flat = s.flatten()
    v = flat.verts.astype(np.float64)[flat.tris.astype(np.int64)]
    n = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    first = s.base.n_tris
    sizes = np.diff(s.mesh_tri_begin.astype(np.int64))
    assert np.linalg.det(s.inst_xform[0].astype(np.float64).reshape(3, 4)[:, :3]) < 0  # the mirrored one
    for j in range(len(s.inst_mesh)):
        cnt = int(sizes[s.inst_mesh[j]])
        x = s.inst_xform[j].astype(np.float64).reshape(3, 4)
        # the meshes are convex around their object-space centroid: outward normals point away
        # from the image of that centroid
        mv = s.mesh_verts.astype(np.float64)
        beg = int(s.mesh_tri_begin[s.inst_mesh[j]])
        c_obj = mv[s.mesh_tris[beg:beg + cnt].astype(np.int64).reshape(-1)].mean(0)
        c = x[:, :3] @ c_obj + x[:, 3]
        cen = v[first:first + cnt].mean(1)
        side = np.sign(np.linalg.det(x[:, :3]))
        assert np.all(side * np.einsum("ij,ij->i", n[first:first + cnt], cen - c) > 0), j
        first += cnt


def test_flatten_evaluates_the_map_in_the_stated_order(scenes):
    # world = ((a00 x + a01 y) + a02 z) + t0 in float64, rounded to float32: the renderer's
    # host code builds the light list and the scene bounds from the same numbers
    s = scenes.instance_field(3, 8)
    flat = s.flatten()
    j = 5
    x = s.inst_xform[j].astype(np.float64).reshape(3, 4)
    m = int(s.inst_mesh[j])
    beg = s.mesh_tri_begin.astype(np.int64)
    first = s.base.n_tris + int(np.diff(beg)[s.inst_mesh[:j]].sum())
    t0 = s.mesh_tris[beg[m]].astype(np.int64)
    for q in range(3):
        p = s.mesh_verts[t0[q]].astype(np.float64)
        want = np.array([np.float32(((x[a, 0] * p[0] + x[a, 1] * p[1]) + x[a, 2] * p[2]) + x[a, 3]) for a in range(3)])
        got = flat.verts[flat.tris[first, q]]
        assert np.array_equal(got, want)


def test_yaw_box_map_is_the_box_construction(scenes):
    # the instanced terrain uses the same map as the flattened terrain's box(): a rotation about
    # +y times the box size, then the centre
    xf = scenes._yaw_box_xform((1.0, 2.0, 3.0), (0.2, 0.4, 0.6), math.radians(30.0)).reshape(3, 4)
    rot = np.array([[math.cos(math.radians(30.0)), 0.0, math.sin(math.radians(30.0))], [0.0, 1.0, 0.0],
                    [-math.sin(math.radians(30.0)), 0.0, math.cos(math.radians(30.0))]])
    corner = np.array([0.5, -0.5, 0.5])
    assert np.allclose(xf[:, :3] @ corner + xf[:, 3], (corner * [0.2, 0.4, 0.6]) @ rot.T + [1.0, 2.0, 3.0])
