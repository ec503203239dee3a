"""The C-ABI library builds, loads and exports every entry point that
include/qhp.h declares (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "qhp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(qhp_\w+)\s*\(", text, re.M)))


def test_header_declares_the_verbs():
    names = declared_symbols()
    for verb in ("qhp_create", "qhp_mesh", "qhp_assemble", "qhp_set_incident", "qhp_step", "qhp_run",
                 "qhp_history_sum", "qhp_destroy"):
        assert verb in names


def test_library_exports_every_declared_symbol():
    import paper_2312_06367_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libqhp.so not built")
    L = ctypes.CDLL(pkg.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert set(declared_symbols()) == set(pkg.EXPORTS)


def test_batch_tile_shape_counts():
    """qhp_batch_variants is host logic: six history tile shapes for FP32 or
    FP32-block/FP64-sum batches with 2, 4 or 8 right-hand sides, one where
    there is no choice, none for unsupported precisions or counts."""
    import paper_2312_06367_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libqhp.so not built")
    for p in ("f32", "f32a"):
        for n in (2, 4, 8):
            assert pkg.batch_variants(p, n) == 6
        assert pkg.batch_variants(p, 1) == 1
        assert pkg.batch_variants(p, 3) == 0
    assert pkg.batch_variants("f64", 8) == 1
    assert pkg.batch_variants("bf16", 4) == 0
    assert pkg.batch_variants("i8x4", 8) == 0


# entry points whose first argument is a handle, with the other arguments
# they take (all passed as zero / null)
_HANDLE_CALLS = {
    "qhp_keep_raw": 1, "qhp_mesh": 4, "qhp_assemble": 0, "qhp_set_precision": 1, "qhp_t0_condition": 3,
    "qhp_set_solver": 1, "qhp_release_assembly": 0, "qhp_profile": 1, "qhp_hist_time": 2,
    "qhp_band_time": 3,
    "qhp_set_incident": 3, "qhp_step": 1, "qhp_run": 3, "qhp_query": 1, "qhp_edges": 2, "qhp_get_matrix": 3,
    "qhp_batch_run": 2, "qhp_batch_step_times": 2, "qhp_set_gmres": 4, "qhp_gmres_stats": 4,
    "qhp_gmres_reset": 0, "qhp_mlp_create": 3, "qhp_mlp_dims": 3, "qhp_mlp_set_params": 1,
    "qhp_mlp_get_params": 1, "qhp_mlp_features": 3, "qhp_mlp_guess": 2, "qhp_mlp_reconstruct": 3,
    "qhp_mlp_forward": 3, "qhp_mlp_loss_grad": 5, "qhp_mlp_adam": 4, "qhp_mlp_train": 7, "qhp_attach_mlp": 1,
}


def test_null_handles_and_bad_sizes_are_rejected():
    """Host logic of the boundary, no device touched: every call on a null
    handle returns QHP_EINVAL and the destroy calls accept one; the history
    sum rejects bad sizes, layouts, ring shapes and variants before it
    allocates or launches anything."""
    import paper_2312_06367_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libqhp.so not built")
    L = ctypes.CDLL(pkg.LIB_PATH)
    EINVAL = -1
    declared = set(declared_symbols())
    for name, nargs in _HANDLE_CALLS.items():
        assert name in declared, name
        f = getattr(L, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p] + [ctypes.c_int64] * nargs
        assert f(None, *([0] * nargs)) == EINVAL, name
    for name in ("qhp_destroy", "qhp_batch_destroy", "qhp_mlp_destroy"):
        f = getattr(L, name)
        f.argtypes = [ctypes.c_void_p]
        f.restype = None
        f(None)
    f = L.qhp_create
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert f(None, None) == EINVAL

    h = L.qhp_history_sum_variant
    h.restype = ctypes.c_int
    h.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    P = {"f64": 0, "f32": 1, "bf16": 2, "f32a": 3, "bf16x2": 4, "i8x4": 5}
    assert [pkg.PRECISIONS[k] for k in P] == list(P.values())
    fake = 4096  # never dereferenced: every case below fails its checks first
    good = dict(p=P["f32"], ne=100, ld=128, nrhs=1, kmax=4, slabs=fake, scales=None, ring=fake, n_slots=4, head=0,
                r=fake, b=fake, variant=-1)
    bad = [dict(ne=0), dict(ld=96), dict(ld=100), dict(nrhs=0), dict(kmax=-1), dict(n_slots=3), dict(head=-1),
           dict(slabs=None), dict(ring=None), dict(r=None), dict(b=None), dict(variant=11), dict(variant=-2),
           dict(p=6), dict(p=-1), dict(p=P["f32a"], nrhs=2), dict(p=P["bf16x2"], nrhs=1),
           dict(p=P["bf16x2"], nrhs=2, ld=136), dict(p=P["i8x4"], nrhs=1), dict(p=P["i8x4"], nrhs=2, ld=160),
           dict(p=P["bf16"], nrhs=1), dict(p=P["f64"], nrhs=2, variant=1)]
    for change in bad:
        a = dict(good, **change)
        rc = h(None, a["p"], a["ne"], a["ld"], a["nrhs"], a["kmax"], a["slabs"], a["scales"], a["ring"],
               a["n_slots"], a["head"], a["r"], a["b"], a["variant"])
        assert rc == EINVAL, change


def _lib_or_skip():
    import paper_2312_06367_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libqhp.so not built")
    return pkg


def test_check_mesh_accepts_closed_surfaces_and_counts_loops():
    """qhp_check_mesh (host only): a closed sphere has N_H = 0 global loops,
    a torus N_H = 2 (Sec. II-D: N_H = 2 - Euler characteristic)."""
    pkg = _lib_or_skip()
    from workloads import meshes
    xyz, tri = meshes.icosphere(1)
    assert pkg.check_mesh(xyz, tri)[:3] == (0, 120, 0)
    xyz, tri = meshes.torus(1.0, 0.3, 12, 5)
    rc, ne, nh, _ = pkg.check_mesh(xyz, tri)
    assert (rc, ne, nh) == (0, 3 * 12 * 5, 2)


def test_check_mesh_rejects_what_the_formulation_excludes():
    """Every mesh the formulation excludes (Sec. II-A: Gamma closed, connected
    and orientable; the bases need non-degenerate triangles) returns
    QHP_EMESH with its reason, before any device work."""
    pkg = _lib_or_skip()
    from workloads import meshes
    EMESH, EINVAL = -2, -1
    xyz, tri = meshes.icosphere(1)
    nv = len(xyz)
    cases = {}
    cases["open"] = (xyz, tri[1:])
    cases["flipped"] = (xyz, np.concatenate([tri[:1, ::-1], tri[1:]]))
    # two separate spheres
    cases["disconnected"] = (np.concatenate([xyz, xyz + 3.0]), np.concatenate([tri, tri + nv]))
    # vertex 0 and its antipode merged into one: every edge still has two
    # consistently oriented triangles, but the triangles at vertex 0 form two discs
    opp = int(np.argmin(np.linalg.norm(xyz + xyz[0], axis=1)))
    keep = np.array([v for v in range(nv) if v != opp])
    renum = np.full(nv, -1)
    renum[keep] = np.arange(nv - 1)
    renum[opp] = 0
    cases["non-manifold vertex"] = (xyz[keep], renum[tri].astype(np.int32))
    # a triangle whose three vertices are collinear: move vertex a onto the
    # midpoint of the other two vertices of one of its triangles
    a, b, c = tri[0]
    xz = xyz.copy()
    xz[a] = 0.5 * (xyz[b] + xyz[c])
    cases["zero area"] = (xz, tri)
    bad = tri.copy()
    bad[0, 1] = bad[0, 0]
    cases["repeated vertex"] = (xyz, bad)
    bad = tri.copy()
    bad[0, 0] = nv
    cases["index out of range"] = (xyz, bad)
    expect = {"open": "exactly two", "flipped": "oriented", "disconnected": "not connected",
              "non-manifold vertex": "non-manifold vertex", "zero area": "zero-area",
              "repeated vertex": "degenerate", "index out of range": "out of range"}
    for name, (x, t) in cases.items():
        rc, _, _, msg = pkg.check_mesh(x, t)
        assert rc == EMESH, (name, rc, msg)
        assert expect[name] in msg, (name, msg)
    L = pkg.lib()
    assert L.qhp_check_mesh(None, 4, None, 4, None, None, None, 0) == EINVAL


def test_allocator_hook_and_growth_limit_argument_checks():
    """Host logic, no device: qhp_create refuses an allocator hook with only
    one of dev_alloc / dev_free; qhp_set_growth_limit rejects a null context."""
    pkg = _lib_or_skip()
    L = pkg.lib()
    p = pkg._Params(0.1, 1.0, 0, 0, 10, 0, None)
    alloc = pkg.TorchAllocator(0)
    p.dev_alloc = alloc.alloc_fn  # dev_free left NULL
    h = ctypes.c_void_p()
    assert L.qhp_create(ctypes.byref(p), ctypes.byref(h)) == -1
    assert not h.value
    assert L.qhp_set_growth_limit(None, 1.0) == -1


def test_temporal_order_argument_check():
    """Host logic, no device: qhp_create takes temporal order 0 / 1 (hat
    functions) and 2 (quadratic interpolators) and refuses others."""
    pkg = _lib_or_skip()
    L = pkg.lib()
    for bad in (-1, 3, 7):
        p = pkg._Params(0.1, 1.0, 0, 0, 10, 0, None)
        p.temporal_order = bad
        h = ctypes.c_void_p()
        assert L.qhp_create(ctypes.byref(p), ctypes.byref(h)) == -1
        assert not h.value


def test_noalloc_history_sum_refuses_before_any_device_work():
    """qhp_history_sum_noalloc (host logic, no device): partial sums beyond
    its fixed array, and the argument errors of the allocating call, return
    QHP_EINVAL; the pointers are never dereferenced."""
    pkg = _lib_or_skip()
    L = pkg.lib()
    hdr = open(os.path.join(ROOT, "include", "qhp.h")).read()
    limit = int(re.search(r"#define QHP_NOALLOC_SCRATCH_MB (\d+)", hdr).group(1)) << 20
    fake = ctypes.c_void_p(4096)
    # 8192 rows x 2048 right-hand sides: even one lag split needs 128 MiB of
    # FP64 partial sums, above the array whatever the split count
    ne, nrhs = 8192, 2048
    assert ne * nrhs * 8 > limit
    f = L.qhp_history_sum_noalloc
    assert f(None, pkg.QHP_F32, ne, ne, nrhs, 4, fake, None, fake, 4, 0, fake, fake, -1) == -1
    assert f(None, pkg.QHP_F32A, 100, 100, 1, 4, fake, None, fake, 4, 0, fake, fake, -1) == -1  # ld % 8
    assert f(None, pkg.QHP_F32, 100, 128, 1, 4, fake, None, fake, 3, 0, fake, fake, -1) == -1  # slots < lags
    assert f(None, pkg.QHP_F32, 100, 128, 1, 4, fake, None, fake, 4, 0, fake, fake, 11) == -1  # variant
