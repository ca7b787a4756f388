"""The C ABI without a GPU: every symbol that include/wos.h declares is exported by libwos.so and
bound by the Python binding, and the host-only entry points (element table, validation, errors)
behave as documented."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.special

import wos_inputs as wi
from oracle import walks as ow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wos.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:wos_status|const\s+char\s*\*)\s*(wos_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def wos():
    from paper_2409_03686_amd import wos as w
    return w


def test_every_declared_symbol_is_exported_and_bound(wos):
    names = _declared()
    assert len(names) >= 19, names
    L = wos.lib()
    for n in names:
        assert hasattr(L, n), f"{n} is declared in wos.h but not exported"
        assert n in wos._SIGS, f"{n} has no binding"


def _geoms():
    return [
        wi.Geometry(2, wi.DISK, (0.1, -0.2, 1.5), (48,)),
        wi.Geometry(2, wi.ANNULUS, (0.0, 0.0, 0.3, 1.0), (128, 128)),
        wi.Geometry(2, wi.ELLIPSE, (0.0, 0.0, 1.0, 0.4), (96,)),
        wi.Geometry(2, wi.POLYGON, (), (60,), verts=wi.L_SHAPE.copy()),
        wi.Geometry(3, wi.BALL, (0.0, 0.0, 0.0, 1.0), (8, 16)),
        wi.Geometry(2, wi.BOX, (0.0, 0.0, 2.0, 1.0), (10,)),
        wi.Geometry(3, wi.BOX, (0.0, 0.0, 0.0, 1.0, 1.0, 1.0), (24,)),
        wi.perforated_disk_example().geom,
        wi.square_hole_example(1).geom,
        wi.spherical_shell_example(7).geom,
        wi.spherical_shell_example(6, outer=(25, 40), inner=(10, 10)).geom,
        wi.Geometry(3, wi.PERFBOX, (0.0, 0.0, 0.0, 1.0, 2.0, 1.0), (6, 4, 5),
                    verts=np.array([[0.3, 0.5, 0.5, 0.2], [0.6, 1.4, 0.5, 0.25]])),
        wi.Geometry(3, wi.PERFBOX, (0.0, 0.0, 0.0, 1.0, 2.0, 1.0), (6, 64, 0),
                    verts=np.array([[0.3, 0.5, 0.5, 0.2], [0.6, 1.4, 0.5, 0.25]])),
        wi.Geometry(3, wi.BALL, (0.0, 0.0, 0.0, 1.3), (2000, 0)),
        wi.Geometry(3, wi.TRIMESH, (), (2,), verts=wi.box_mesh([0.0, 0.0, 0.0], [1.0, 2.0, 0.5], 5)),
        wi.Geometry(3, wi.TRIMESH, (), (1,), verts=wi.sphere_mesh([0.1, 0.0, 0.0], 0.7, 2)),
        wi.Geometry(3, wi.TRIMESH, (), (4,), verts=wi.l_prism_mesh(4)),
    ]


def test_element_table_matches_oracle(wos):
    for g in _geoms():
        n = wos.wos_element_count(g)
        assert n == g.n_elem
        s = wos.wos_element_measures(g)
        so = ow.element_measures(g)
        # Voronoi cells of Bauer nodes: the library's clipped polygons against scipy's diagram
        np.testing.assert_allclose(s, so, rtol=1e-9 if 0 in tuple(g.layout) else 1e-12, atol=0)


def test_oracle_ellipse_cells_sum_to_the_perimeter():
    """Pin of the oracle's Gauss-Legendre cell measures: their sum is the ellipse perimeter
    4 a E(1 - b^2/a^2) (complete elliptic integral of the second kind)."""
    a, b = 1.0, 0.4
    g = wi.Geometry(2, wi.ELLIPSE, (0.0, 0.0, a, b), (96,))
    per = 4 * a * scipy.special.ellipe(1 - (b / a) ** 2)
    assert abs(ow.element_measures(g).sum() - per) < 1e-12 * per


def test_invalid_geometries_are_rejected_on_the_host(wos):
    bad = [
        (wi.Geometry(2, wi.DISK, (0.0, 0.0, -1.0), (8,)), wos.WOS_EINVAL),
        (wi.Geometry(3, wi.DISK, (0.0, 0.0, 1.0), (8,)), wos.WOS_EINVAL),
        (wi.Geometry(2, wi.ANNULUS, (0.0, 0.0, 1.0, 0.5), (8, 8)), wos.WOS_EINVAL),
        (wi.Geometry(2, wi.POLYGON, (), (8,), verts=wi.L_SHAPE[::-1].copy()), wos.WOS_EINVAL),  # clockwise
        (wi.Geometry(2, wi.POLYGON, (), (8,), verts=wi.L_SHAPE[:2].copy()), wos.WOS_EINVAL),    # 2 vertices
        (wi.Geometry(3, wi.BOX, (0.0, 0.0, 0.0, 1.0, 0.0, 1.0), (4,)), wos.WOS_EINVAL),         # lo == hi
        (wi.Geometry(2, 9, (0.0, 0.0, 1.0), (8,)), wos.WOS_EINVAL),                            # unknown kind
        (wi.Geometry(2, wi.DISK, (0.0, 0.0, 1.0), (16385,)), wos.WOS_ENOTSUP),                 # too many cells
        (wi.Geometry(2, wi.DISK, (0.0, 0.0, float("nan")), (8,)), wos.WOS_EINVAL),
        (wi.Geometry(2, wi.PERFORATED, (0.0, 0.0, 1.0), (8, 4, 1), verts=np.array([[0.7, 0.0, 0.4]])),
         wos.WOS_EINVAL),                                                                      # hole sticks out
        (wi.Geometry(2, wi.PERFORATED, (0.0, 0.0, 1.0), (8, 4, 2), verts=np.array([[0.2, 0.0, 0.3], [-0.2, 0.0, 0.3]])),
         wos.WOS_EINVAL),                                                                      # holes overlap
        (wi.Geometry(2, wi.PERFORATED, (0.0, 0.0, 1.0), (8, 4, 2), verts=np.array([[0.2, 0.0, 0.1]])),
         wos.WOS_EINVAL),                                                                      # 1 hole given, 2 declared
        (wi.Geometry(3, wi.PERFORATED, (0.0, 0.0, 0.0, 1.0), (4, 8, 2, 4), verts=np.array([[0.0, 0.0, 0.6, 0.5]])),
         wos.WOS_EINVAL),                                                                      # hole sticks out
        (wi.Geometry(3, wi.PERFORATED, (0.0, 0.0, 0.0, 1.0), (4, 8, 0, 4), verts=np.array([[0.0, 0.0, 0.0, 0.5]])),
         wos.WOS_EINVAL),                                                                      # no hole cells
        (wi.Geometry(2, wi.PERFBOX, (-1.0, -1.0, 1.0, 1.0), (4, 8), verts=np.array([[0.9, 0.0, 0.2]])),
         wos.WOS_EINVAL),                                                                      # hole crosses a face
        (wi.Geometry(2, wi.PERFBOX, (-1.0, -1.0, 1.0, 1.0), (4, 8), verts=np.array([[0.0, 0.0, -0.2]])),
         wos.WOS_EINVAL),                                                                      # r < 0
        (wi.Geometry(3, wi.PERFBOX, (0.0, 0.0, 0.0, 1.0, 1.0, 1.0), (4, 8), verts=np.array([[0.5, 0.5, 0.5, 0.2]])),
         wos.WOS_EINVAL),                                                                      # 3D hole cells missing
        (wi.Geometry(3, wi.BALL, (0.0, 0.0, 0.0, 1.0), (8, 0)), wos.WOS_EINVAL),                # < 16 Bauer nodes
        (wi.Geometry(3, wi.TRIMESH, (), (5,), verts=wi.box_mesh([0, 0, 0], [1, 1, 1], 1)), wos.WOS_EINVAL),  # 5 does not divide 12
        (wi.Geometry(3, wi.TRIMESH, (), (1,), verts=wi.box_mesh([0, 0, 0], [1, 1, 1], 1)[:3]), wos.WOS_EINVAL),  # < 4 triangles
        (wi.Geometry(3, wi.TRIMESH, (), (1,), verts=np.concatenate(
            [wi.box_mesh([0, 0, 0], [1, 1, 1], 1), [[[0, 0, 0], [1, 1, 1], [2, 2, 2]]]])), wos.WOS_EINVAL),  # degenerate
        (wi.Geometry(2, wi.TRIMESH, (), (1,), verts=wi.box_mesh([0, 0, 0], [1, 1, 1], 1)), wos.WOS_EINVAL),  # dim 2
    ]
    for g, code in bad:
        with pytest.raises(wos.WosError) as e:
            wos.wos_element_count(g)
        assert e.value.status == code, (g, e.value)
        assert len(str(e.value)) > 0


def test_context_creation_reports_a_missing_device(wos):
    L = wos.lib()
    p = C.c_void_p()
    st = L.wos_create(C.byref(p), 0, 0)
    if st == wos.WOS_OK:  # a GPU is present: nothing to check here
        L.wos_destroy(p)
        pytest.skip("a GPU is present")
    assert st == wos.WOS_EDEVICE
    assert b"device" in L.wos_last_error()


def test_null_arguments_are_rejected(wos):
    L = wos.lib()
    assert L.wos_element_count(None, None) == wos.WOS_EINVAL
    assert L.wos_plan_destroy(None) in (wos.WOS_OK, wos.WOS_EINVAL)
    # the products reject missing arguments before touching a device
    assert L.wos_density(None, None, 1, 1, 1, None, None, None, None) == wos.WOS_EINVAL
    assert L.wos_eigenfunctions(None, None, 0, None, None, None) == wos.WOS_EINVAL
    assert L.wos_reconstruct_sweep(None, None, None, 1, None, None, 1, None, None, None, None) == wos.WOS_EINVAL
