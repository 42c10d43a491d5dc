"""The seeded synthetic inputs against the configurations they stand for
(CPU only): lattice shapes, electrode layout and potentials, salt from the
Debye length, applied fields, noise amplitude and seeding, the sphere
packing of the porous electrode and the parameter ranges of the batch."""
import math

import numpy as np
import pytest

import workloads as W


def debye_length(z, n, lB):
    """lambda_D = (4 pi l_B sum_k z_k^2 n_k)^(-1/2), written from the species
    sum rather than the 1:1 shortcut the generators use."""
    return 1.0 / math.sqrt(4.0 * math.pi * lB * sum(zk * zk * nk for zk, nk in zip(z, n)))


def check_noise(w, rel):
    fluid = w.node_type == 0
    assert (w.n_init[:, ~fluid] == 0).all()
    for k, ref in enumerate(w.n_ref):
        dev = w.n_init[k, fluid] / ref - 1.0
        assert np.abs(dev).max() <= rel * (1 + 1e-9)
        assert np.abs(dev).max() >= 0.9 * rel  # uniform in [-rel, rel]: the edge is reached
        assert abs(dev.mean()) <= 0.05 * rel


def slab_planes(w):
    nx, ny, nz = w.shape
    return w.node_type.reshape(nz, ny, nx), w.phi_s.reshape(nz, ny, nx)


def test_salt_from_debye_length():
    for debye in (2.0, 4.0, 6.0, 8.0, 16.0):
        rs = W.salt_for_debye(debye, 0.4)
        assert debye_length((1, -1), (rs, rs), 0.4) == pytest.approx(debye, rel=1e-14)


def test_parallel_plate_capacitor():
    w = W.parallel_plate_small()
    assert w.shape == (4, 4, 34)
    t, ps = slab_planes(w)
    assert (t[0] == 1).all() and (ps[0] == 0.05).all()
    assert (t[33] == 2).all() and (ps[33] == -0.05).all()
    assert (t[1:33] == 0).all() and (ps[1:33] == 0).all()
    assert debye_length(w.z, w.n_ref, w.lB) == pytest.approx(4.0)
    assert (w.lB, w.tau, w.D, w.omega, w.tol, w.steps) == (0.4, 1.0, (0.05, 0.05), 1.8, 1e-10, 20000)
    check_noise(w, 1e-6)
    assert np.array_equal(w.n_init, W.parallel_plate_small().n_init)  # seeded


def test_electro_osmosis_slab():
    w = W.eo_slab()
    assert w.shape == (64, 64, 130)
    t, ps = slab_planes(w)
    assert (t[0] == 1).all() and (ps[0] == 0.1).all()
    assert (t[129] == 2).all() and (ps[129] == -0.1).all()
    assert (t[1:129] == 0).all()
    assert debye_length(w.z, w.n_ref, w.lB) == pytest.approx(8.0)
    assert w.Eapp == (1e-3, 0.0, 0.0) and w.steps == 50000
    check_noise(w, 1e-6)
    # its own noise stream, not the capacitor's: the relative deviations of
    # the first fluid plane differ
    c = W.parallel_plate_small()
    dw = w.n_init[0, 64 * 64:64 * 64 + 16] / w.n_ref[0]
    dc = c.n_init[0, 16:32] / c.n_ref[0]
    assert not np.array_equal(dw, dc)


def test_coaxial_cell():
    w = W.coaxial()
    assert w.shape == (160, 160, 64)
    r = W.radial_distance(w.shape)
    t = w.node_type
    assert ((t == 1) == (r < 8.0)).all() and ((t == 2) == (r > 72.0)).all()
    assert (w.phi_s[t == 1] == 0.05).all() and (w.phi_s[t == 2] == -0.05).all()
    # the same cross-section on every plane (periodic along z)
    t3 = t.reshape(64, 160, 160)
    assert (t3 == t3[0]).all()
    # fluid per plane: the annulus 8 <= r <= 72 of the staircase, close to
    # its continuous area
    nf = int((t3[0] == 0).sum())
    assert abs(nf - math.pi * (72.0 ** 2 - 8.0 ** 2)) / nf < 0.01
    assert debye_length(w.z, w.n_ref, w.lB) == pytest.approx(6.0)
    assert w.tau == 0.8 and w.Eapp == (0.0, 0.0, 1e-3) and w.steps == 30000
    check_noise(w, 1e-6)


@pytest.fixture(scope="module")
def porous():
    return W.porous_electrode()


def test_porous_electrode_packing(porous):
    """Spheres of radius 6-10 at +0.05 in z = 16..159 filling 28-30% of that
    slab (random sequential addition stops near 28.4% when no sphere fits),
    nothing solid in the gap z = 160..175, a flat counter-electrode
    z = 176..191 at -0.05.  Every face-connected solid component of the
    packing, joined across the periodic x and y faces, has the voxel count of
    one ball of radius 6 to 10: no two spheres overlap or share a face."""
    import scipy.ndimage as nd
    w = porous
    assert w.shape == (192, 192, 192)
    t3 = w.node_type.reshape(192, 192, 192)
    p3 = w.phi_s.reshape(192, 192, 192)
    assert (t3[:16] == 0).all() and (t3[160:176] == 0).all()
    assert (t3[176:] == 2).all() and (p3[176:] == -0.05).all()
    slab = t3[16:160]
    assert set(np.unique(slab).tolist()) == {0, 1}
    assert (p3[16:160][slab == 1] == 0.05).all()
    frac = (slab == 1).mean()
    assert 0.28 <= frac <= 0.30
    assert debye_length(w.z, w.n_ref, w.lB) == pytest.approx(4.0)
    check_noise(w, 1e-6)

    lab, n = nd.label(slab == 1)
    parent = np.arange(n + 1)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for ax in (1, 2):  # y and x faces
        a, b = np.take(lab, 0, axis=ax), np.take(lab, -1, axis=ax)
        both = (a > 0) & (b > 0)
        for x, y in set(zip(a[both].tolist(), b[both].tolist())):
            rx, ry = find(x), find(y)
            if rx != ry:
                parent[rx] = ry
    sizes = np.bincount(lab.ravel())[1:]
    roots = np.array([find(i) for i in range(1, n + 1)])
    balls = np.bincount(roots, weights=sizes)
    balls = balls[balls > 0]
    vol = lambda r: 4.0 / 3.0 * math.pi * r ** 3  # noqa: E731
    assert balls.min() >= 0.95 * vol(6.0) and balls.max() <= 1.02 * vol(10.0)
    # the ball volumes add up to the solid of the slab
    assert balls.sum() == (slab == 1).sum()


def test_porous_crops_are_cut_from_the_electrode(porous):
    t3 = porous.node_type.reshape(192, 192, 192)
    c = W.porous_crop(noise=False)
    assert c.shape == (24, 24, 24)
    assert np.array_equal(c.node_type.reshape(24, 24, 24), t3[156:180, :24, :24])
    col = W.porous_column(noise=False)
    assert col.shape == (32, 32, 192)
    assert np.array_equal(col.node_type.reshape(192, 32, 32), t3[:, :32, :32])


def test_batch_of_plate_systems():
    """96 systems of 8 x 8 x L (L uniform in 16..256), voltages uniform in
    [0.01, 0.2] split +V/2, -V/2 over each system's two electrodes, Debye
    lengths uniform in [2, 16]; each system an even number of planes (one
    bottom electrode plane, L fluid planes, one or two top planes)."""
    b = W.batch_slabs()
    nsys = 96
    assert len(b.L) == len(b.V) == len(b.debye) == nsys
    assert b.L.min() >= 16 and b.L.max() <= 256
    assert b.V.min() >= 0.01 and b.V.max() <= 0.2
    assert b.debye.min() >= 2.0 and b.debye.max() <= 16.0
    # spread over the ranges, not clustered (seeded draws)
    assert b.L.max() - b.L.min() > 180 and b.debye.max() - b.debye.min() > 10
    nx, ny, nz = b.shape
    assert (nx, ny) == (8, 8)
    t3 = b.node_type.reshape(nz, 8, 8)
    p3 = b.phi_s.reshape(nz, 8, 8)
    s3 = b.system.reshape(nz, 8, 8)
    z = 0
    for s in range(nsys):
        planes = b.L[s] + 2 + (b.L[s] % 2)
        assert planes % 2 == 0 and b.z0[s] == z + 1
        assert (t3[z] == 2 * s + 1).all() and np.allclose(p3[z], 0.5 * b.V[s])
        fl = slice(z + 1, z + 1 + b.L[s])
        assert (t3[fl] == 0).all() and (s3[fl] == s).all()
        top = slice(z + 1 + b.L[s], z + planes)
        assert (t3[top] == 2 * s + 2).all() and np.allclose(p3[top], -0.5 * b.V[s])
        assert debye_length(b.z, b.n_ref[s], b.lB) == pytest.approx(b.debye[s])
        z += planes
    assert z == nz
    fluid = b.node_type == 0
    dev = b.n_init[:, fluid] / b.n_ref[b.system[fluid]].T - 1.0
    assert np.abs(dev).max() <= 1e-6 * (1 + 1e-9) and np.abs(dev).max() >= 0.9e-6
    assert (b.n_init[:, ~fluid] == 0).all()
    again = W.batch_slabs()
    assert np.array_equal(again.L, b.L) and np.array_equal(again.n_init, b.n_init)
