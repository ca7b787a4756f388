"""The FP32 cell index of stops on circles (element32_certified in wos_device.hpp) must never
disagree with the FP64 rule where it answers.  Its FP32 arithmetic is replayed here in numpy
(hardware reciprocal modelled as the correctly rounded one moved by up to one ulp) on stop
positions near both circles of an annulus and of a disk, with a quarter of them placed on cell
boundaries, and compared with the FP64 arc rule: floor(theta n / 2 pi) with theta = atan2 shifted
to [0, 2 pi), the circle chosen by the nearer radius."""
import numpy as np

f32 = np.float32
# the kernel's polynomial for atan(a) / 2 pi on [0, 1], highest power of a^2 first
POLY = [0.0010841292096301913, -0.005348275415599346, 0.012672500684857368, -0.021061519160866737,
        0.03152512013912201, -0.053026240319013596, 0.15915432572364807]


def _fma(a, b, c):
    return f32(np.float64(a) * np.float64(b) + np.float64(c))


def _cells32(x, y, n0, n1, annulus, pf6, pf7, rng):
    ax, ay = np.abs(x), np.abs(y)
    mx = np.maximum(ax, ay)
    rcp = (f32(1.0) / mx).astype(f32)
    rcp = np.nextafter(rcp, np.where(rng.random(rcp.shape) < 0.5, f32(np.inf), f32(-np.inf))).astype(f32)
    a = (np.minimum(ax, ay) * rcp).astype(f32)
    z = (a * a).astype(f32)
    p = np.full_like(a, f32(POLY[0]))
    for c in POLY[1:]:
        p = _fma(p, z, f32(c))
    r = (p * a).astype(f32)
    r = np.where(ay > ax, (f32(0.25) - r).astype(f32), r)
    r = np.where(x < 0, (f32(0.5) - r).astype(f32), r)
    r = np.where(y < 0, -r, r)
    r = np.where(r < 0, (r + f32(1)).astype(f32), r)
    n = np.full(x.shape, n0)
    off = np.zeros(x.shape, np.int64)
    undecided = np.zeros(x.shape, bool)
    if annulus:
        rho2 = _fma(x, x, (y * y).astype(f32))
        outer, inner = rho2 >= pf7, rho2 <= pf6
        n = np.where(outer, n0, n1)
        off = np.where(outer, 0, n0)
        undecided = ~(outer | inner)
    nf = n.astype(f32)
    t = (r * nf).astype(f32)
    fl = np.floor(t)
    fr = (t - fl).astype(f32)
    m = (nf * f32(2.0 ** -20)).astype(f32)
    ok = (fr > m) & (fr < f32(1) - m) & ~undecided
    return np.where(ok, off + fl.astype(np.int64), -1)


def _cells64(x, y, n0, n1, annulus, r_in, r_out):
    dx, dy = x.astype(np.float64), y.astype(np.float64)
    two_pi = 6.283185307179586
    th = np.arctan2(dy, dx)
    th = np.where(th < 0, th + two_pi, th)

    def arc(n):
        return np.minimum(np.floor(th * n / two_pi).astype(np.int64), n - 1)

    if not annulus:
        return arc(n0)
    rho = np.sqrt(dx * dx + dy * dy)
    return np.where((r_out - rho) <= (rho - r_in), arc(n0), n0 + arc(n1))


def test_fp32_cells_agree_with_fp64_wherever_accepted():
    rng = np.random.default_rng(3)
    for annulus, (r_in, r_out, n0, n1) in [(True, (0.3, 1.0, 128, 128)), (False, (0.0, 1.5, 48, 0)),
                                          (True, (0.3, 1.0, 2000, 16384))]:
        mid, w = 0.5 * (r_in + r_out), 0.5 * (r_out - r_in)
        pf6, pf7 = f32((mid - 0.25 * w) ** 2), f32((mid + 0.25 * w) ** 2)
        N = 200_000
        th = rng.uniform(0, 2 * np.pi, N)
        k = rng.integers(0, n0, N // 4)
        th[: N // 4] = 2 * np.pi * k / n0 + rng.normal(0, 1e-6, N // 4)  # on cell boundaries
        th[N // 4: N // 4 + 700] = np.repeat([0, np.pi / 4, np.pi / 2, np.pi, 1.5 * np.pi, -1e-9, 1e-9], 100)
        rad = np.where(rng.random(N) < 0.5, r_out, r_in if annulus else r_out) - rng.uniform(0, 1e-4, N)
        x, y = (rad * np.cos(th)).astype(f32), (rad * np.sin(th)).astype(f32)
        x[:100] = f32(-0.0)
        j32 = _cells32(x, y, n0, n1, annulus, pf6, pf7, rng)
        j64 = _cells64(x, y, n0, n1, annulus, r_in, r_out)
        accepted = j32 >= 0
        assert accepted.mean() > 0.7
        assert np.array_equal(j32[accepted], j64[accepted])
