"""Immersed walls in rigid translation (ibm_set_wall_velocity) with the geometry replaced
between steps (ibm_set_geometry), through the C ABI, against the oracle given the same
sequence of signed distances and velocities."""
import math

import numpy as np
import pytest
import torch

import ibm_inputs as I
from oracle.ibm_oracle import CPG, OGrid, Oracle, wall_shear_profile
from tests.gpu_helpers import case, device, gpu_grid, oracle_run, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    device()


def _say(*a):
    print(*a, flush=True)


def _errs(g, o, inst=0):
    u, v, w, p = [t.cpu().numpy() for t in g.get_state(inst=inst)]
    scale = max(np.abs(o.u).max(), np.abs(o.v).max(), np.abs(o.w).max())
    return [np.abs(a - b).max() / scale for a, b in ((u, o.u), (v, o.v), (w, o.w))], (u, v, w, p)


@pytest.mark.parametrize("off", [0.37, 1.37])
def test_sliding_walls_poiseuille(off):
    """Walls sliding along x at U_w: the discrete Poiseuille profile plus U_w stays put on
    the GPU, equal to the oracle's steps."""
    c = I.Case(nx=8, ny=33, nz=4, lx=2 * math.pi, lz=math.pi, y_lo=-1.0, y_hi=1.0, nu=0.01, dt=0.05, forcing=CPG,
               q_target_or_pi=-0.02, geometry="flat", geo_params=(off,))
    g_ = OGrid.from_case(c)
    uw = 0.73
    yc = g_.y_lo + (np.arange(g_.ny - 1) + 0.5) * g_.dy
    hw = 1.0 - off * g_.dy
    inside = np.abs(yc) < hw
    delta = yc[int(np.argmax(inside))] + hw
    a = 0.02 / (2 * g_.nu)
    prof = np.where(inside, a * (hw * hw - yc * yc + delta * (g_.dy - delta)) + uw, uw)
    u = np.broadcast_to(prof[:, None, None], g_.shape).copy()
    z = np.zeros_like(u)
    sdf = I.make_sdf(c)
    o = Oracle(g_)
    o.set_geometry(*sdf)
    o.set_wall_velocity(uw, 0.0, 0.0)
    o.set_state(u, z, z, z)
    o.step(3)
    g = gpu_grid(c, sdf, (u, z, z, z))
    g.set_wall_velocity(uw)
    g.step(3)
    errs, (ug, vg, wg, pg) = _errs(g, o)
    _say(f"off {off}: vs oracle {['%.1e' % e for e in errs]}, drift {np.abs(ug - u).max():.1e}")
    assert max(errs) < 1e-13
    assert np.abs(ug - u).max() < 1e-13 * np.abs(u).max()
    tau, _ = g.wall_shear()
    ref = wall_shear_profile(o.g, o.u, sdf[0], wall_velocity=uw)
    assert np.abs(tau.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    g.close()


def _body_sdf(c, centre, radius):
    """A sphere (minimum image in x and z); the channel walls are the box walls, at rest."""
    def fn(X, Y, Z):
        dx = X - centre[0]
        dx -= c.lx * np.round(dx / c.lx)
        dz = Z - centre[2]
        dz -= c.lz * np.round(dz / c.lz)
        return np.sqrt(dx * dx + (Y - centre[1]) ** 2 + dz * dz) - radius
    return I._sample(c, fn)


@pytest.mark.parametrize("vel", [(0.6, 0.0, 0.0), (0.2, -0.35, 0.15)])
def test_translating_body_against_oracle(vel):
    """A sphere translating through a plane channel: its signed distances at the new
    position and its velocity are given before every step."""
    c = I.Case(nx=32, ny=17, nz=16, lx=2.0, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=0.02, dt=0.01, q_target_or_pi=1.0,
               seed=9, geometry="flat", geo_params=(0.0,))
    g_ = OGrid.from_case(c)
    centre = np.array([0.6, -0.1, 0.45])
    sdf = _body_sdf(c, centre, 0.3)
    u0, v0, w0 = I.laminar_plus_solenoidal(c, sdf, c.seed, amp=0.05)
    st = (u0, v0, w0, np.zeros_like(u0))
    o = Oracle(g_)
    o.set_geometry(*sdf)
    o.set_wall_velocity(*vel)
    o.set_state(*st)
    g = gpu_grid(c, sdf, st)
    g.set_wall_velocity(*vel)
    for n in range(4):
        o.step(1)
        g.step(1)
        errs, _ = _errs(g, o)
        _say(f"vel {vel} step {n + 1}: {['%.1e' % e for e in errs]}")
        assert max(errs) < 1e-12
        centre = centre + np.array(vel) * c.dt
        sdf = _body_sdf(c, centre, 0.3)
        o.set_geometry(*sdf)
        g.set_geometry(*[to_dev(a) for a in sdf])
    assert g.stats()["n_ibm"][0] > 0
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_geometry_update_applies_the_pending_projection(precision):
    """A geometry update right after a step applies the step's pending projection with the
    old tags in its first kernel: the same, bit for bit, as taking the state out and
    seeding it back before the update (nothing pending then); and, moving a sphere each
    step, the oracle's trajectory (FP64 to 1e-12, FP32 storage to 1e-5)."""
    c = I.Case(nx=32, ny=17, nz=16, lx=2.0, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=0.02, dt=0.01, q_target_or_pi=1.0,
               seed=9, geometry="flat", geo_params=(0.0,))
    vel = (0.2, -0.35, 0.15)
    centre = np.array([0.6, -0.1, 0.45])
    sdf = _body_sdf(c, centre, 0.3)
    u0, v0, w0 = I.laminar_plus_solenoidal(c, sdf, c.seed, amp=0.05)
    st = (u0, v0, w0, np.zeros_like(u0))
    o = Oracle(OGrid.from_case(c))
    o.set_geometry(*sdf)
    o.set_wall_velocity(*vel)
    o.set_state(*st)
    a = gpu_grid(c, sdf, st, precision=precision)
    b = gpu_grid(c, sdf, st, precision=precision)
    for g in (a, b):
        g.set_wall_velocity(*vel)
    for n in range(3):
        o.step(1)
        a.step(1)
        b.step(1)
        b.set_state(*b.get_state())           # b: the projection applied and seeded back
        centre = centre + np.array(vel) * c.dt
        sdf = _body_sdf(c, centre, 0.3)
        o.set_geometry(*sdf)
        a.set_geometry(*[to_dev(x) for x in sdf])   # a: applied inside the update
        b.set_geometry(*[to_dev(x) for x in sdf])
    o.step(1)
    a.step(1)
    b.step(1)
    sa, sb = a.get_state(), b.get_state()
    for x, y in zip(sa, sb):
        assert torch.equal(x, y)
    errs, _ = _errs(a, o)
    _say(f"{precision}: after 3 moves {['%.1e' % e for e in errs]}")
    assert max(errs) < (1e-12 if precision == "fp64" else 1e-5)
    a.close()
    b.close()


def test_many_geometry_updates_keep_the_oracle_trajectory():
    """Thirty moves of the sphere in a row, the library's step graph on, with no state read
    in between: every update's flow-rate coefficients S_k come from the last list block to
    finish (a device counter that each update must leave at zero), so a stale or missed S_k
    anywhere would show in the flow rate and the state after the last step."""
    c = I.Case(nx=32, ny=17, nz=16, lx=2.0, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=0.02, dt=0.01, q_target_or_pi=1.0,
               seed=9, geometry="flat", geo_params=(0.0,))
    vel = (0.5, 0.1, -0.2)
    centre = np.array([0.6, -0.2, 0.45])
    sdf = _body_sdf(c, centre, 0.3)
    u0, v0, w0 = I.laminar_plus_solenoidal(c, sdf, c.seed, amp=0.05)
    st = (u0, v0, w0, np.zeros_like(u0))
    o = Oracle(OGrid.from_case(c))
    o.set_geometry(*sdf)
    o.set_wall_velocity(*vel)
    o.set_state(*st)
    g = gpu_grid(c, sdf, st)
    g.set_wall_velocity(*vel)
    g.tune(graph=1)
    for n in range(30):
        o.step(1)
        g.step(1)
        centre = centre + np.array(vel) * c.dt
        sdf = _body_sdf(c, centre, 0.3)
        o.set_geometry(*sdf)
        g.set_geometry(*[to_dev(a) for a in sdf])
    o.step(1)
    g.step(1)
    errs, _ = _errs(g, o)
    _say(f"30 moves: {['%.1e' % e for e in errs]}")
    assert max(errs) < 1e-12
    s = g.stats()
    assert s["n_ibm"][0] > 0 and s["nan_flag"] == 0
    g.close()


def test_zero_wall_velocity_is_bitwise_the_plain_step():
    c = case("wavy_small")
    o, sdf, st = oracle_run(c, 0)
    a = gpu_grid(c, sdf, st)
    b = gpu_grid(c, sdf, st)
    b.set_wall_velocity(0.0, 0.0, 0.0)
    a.step(2)
    b.step(2)
    for x, y in zip(a.get_state(), b.get_state()):
        assert torch.equal(x, y)
    a.close()
    b.close()


def test_moving_instance_in_a_graph_ensemble():
    """An ensemble with one sliding-wall instance, stepped as a HIP graph of batched
    launches (rebuilt after the velocity is set), equals both oracle runs."""
    from paper_2506_14328_amd import IbmGrid
    cs = [case("wavy_small"), case("open_small")]
    runs = [oracle_run(x, 0) for x in cs]
    g = IbmGrid.ensemble(cs, precision="fp64")
    for i, (o, sdf, st) in enumerate(runs):
        g.set_geometry(*[to_dev(a) for a in sdf], inst=i)
        g.set_state(*[to_dev(a) for a in st], inst=i)
    g.tune(graph=1, batch=1)
    g.step(1)
    runs[0][0].step(1)
    runs[1][0].step(1)
    runs[1][0].set_wall_velocity(0.3, 0.0, 0.0)
    g.set_wall_velocity(0.3, inst=1)
    g.step(2)
    runs[0][0].step(2)
    runs[1][0].step(2)
    for i, (o, sdf, st) in enumerate(runs):
        errs, _ = _errs(g, o, inst=i)
        _say(f"instance {i}: {['%.1e' % e for e in errs]}")
        assert max(errs) < 1e-12
    g.close()


def test_translating_body_on_stretched_grid():
    """The translating sphere on tanh-clustered wall-normal faces: sigma and lambda from
    the stretched arms, the geometry replaced every step."""
    import dataclasses
    c = I.Case(nx=32, ny=17, nz=16, lx=2.0, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=0.02, dt=0.01, q_target_or_pi=1.0,
               seed=9, geometry="flat", geo_params=(0.0,))
    c = dataclasses.replace(c, y_faces=I.tanh_faces(c.ny, c.y_lo, c.y_hi, 1.2))
    vel = (0.3, 0.2, -0.1)
    centre = np.array([0.6, -0.1, 0.45])
    sdf = _body_sdf(c, centre, 0.3)
    u0, v0, w0 = I.laminar_plus_solenoidal(c, sdf, c.seed, amp=0.05)
    st = (u0, v0, w0, np.zeros_like(u0))
    o = Oracle(OGrid.from_case(c))
    o.set_geometry(*sdf)
    o.set_wall_velocity(*vel)
    o.set_state(*st)
    g = gpu_grid(c, sdf, st)
    g.set_wall_velocity(*vel)
    for n in range(3):
        o.step(1)
        g.step(1)
        errs, _ = _errs(g, o)
        _say(f"stretched, vel {vel} step {n + 1}: {['%.1e' % e for e in errs]}")
        assert max(errs) < 1e-12
        centre = centre + np.array(vel) * c.dt
        sdf = _body_sdf(c, centre, 0.3)
        o.set_geometry(*sdf)
        g.set_geometry(*[to_dev(a) for a in sdf])
    g.close()


def test_translating_body_with_masked_projection():
    """The translating sphere with continuity imposed on the internal cells only (the
    masked projection): external faces hold the body's velocity, whose net flux through
    the closed staircase surface is zero, so the masked system stays consistent."""
    import dataclasses
    c = I.Case(nx=32, ny=17, nz=16, lx=2.0, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=0.02, dt=0.01, q_target_or_pi=1.0,
               seed=9, geometry="flat", geo_params=(0.0,))
    c = dataclasses.replace(c, projection=1)
    vel = (0.4, -0.2, 0.1)
    centre = np.array([0.6, -0.1, 0.45])
    sdf = _body_sdf(c, centre, 0.3)
    u0, v0, w0 = I.laminar_plus_solenoidal(c, sdf, c.seed, amp=0.05)
    st = (u0, v0, w0, np.zeros_like(u0))
    o = Oracle(OGrid.from_case(c))
    o.set_geometry(*sdf)
    o.set_wall_velocity(*vel)
    o.set_state(*st)
    g = gpu_grid(c, sdf, st)
    g.set_wall_velocity(*vel)
    for n in range(2):
        o.step(1)
        g.step(1)
        errs, _ = _errs(g, o)
        _say(f"masked, vel {vel} step {n + 1}: {['%.1e' % e for e in errs]}")
        assert max(errs) < 1e-11
        centre = centre + np.array(vel) * c.dt
        sdf = _body_sdf(c, centre, 0.3)
        o.set_geometry(*sdf)
        g.set_geometry(*[to_dev(a) for a in sdf])
    g.close()


def _sphere_case():
    return I.Case(nx=32, ny=17, nz=16, lx=2.0, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=0.02, dt=0.01, q_target_or_pi=1.0,
                  seed=9, geometry="flat", geo_params=(0.0,))


def test_translating_body_with_the_graph_on():
    """The translating sphere with the library's HIP graph on: a new geometry with no more
    immersed-boundary points than the lists hold is processed on the stream without a
    host read-back and keeps the captured graph, which then replays each step."""
    c = _sphere_case()
    vel = (0.6, -0.2, 0.1)
    centre = np.array([0.6, -0.1, 0.45])
    sdf = _body_sdf(c, centre, 0.3)
    u0, v0, w0 = I.laminar_plus_solenoidal(c, sdf, c.seed, amp=0.05)
    st = (u0, v0, w0, np.zeros_like(u0))
    o = Oracle(OGrid.from_case(c))
    o.set_geometry(*sdf)
    o.set_wall_velocity(*vel)
    o.set_state(*st)
    g = gpu_grid(c, sdf, st)
    g.set_wall_velocity(*vel)
    g.tune(graph=1)
    for n in range(4):
        o.step(1)
        g.step(1)
        errs, _ = _errs(g, o)
        s = g.stats()
        _say(f"graph, step {n + 1}: {['%.1e' % e for e in errs]}, n_ibm {s['n_ibm']} (oracle "
             f"{[int((o.lam[k] > 0).sum()) for k in 'uvw']})")
        assert max(errs) < 1e-12
        assert s["n_ibm"] == [int((o.lam[k] > 0).sum()) for k in "uvw"]
        centre = centre + np.array(vel) * c.dt
        sdf = _body_sdf(c, centre, 0.3)
        o.set_geometry(*sdf)
        g.set_geometry(*[to_dev(a) for a in sdf])
    g.close()


def test_translating_body_inside_a_caller_graph():
    """A caller captures one move of the body and one step (ibm_set_geometry from
    signed-distance buffers it refills, then ibm_step) into a HIP graph of its own and
    replays it: the geometry update enqueues kernels and copies only (no synchronisation,
    allocation or memset), and every replay equals the oracle's step."""
    import ctypes
    c = _sphere_case()
    vel = (0.5, 0.1, -0.2)
    centre = np.array([0.7, 0.05, 0.4])
    sdf = _body_sdf(c, centre, 0.3)
    u0, v0, w0 = I.laminar_plus_solenoidal(c, sdf, c.seed, amp=0.05)
    st = (u0, v0, w0, np.zeros_like(u0))
    o = Oracle(OGrid.from_case(c))
    o.set_geometry(*sdf)
    o.set_wall_velocity(*vel)
    o.set_state(*st)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = gpu_grid(c, sdf, st)
        g.set_wall_velocity(*vel)
        bufs = [to_dev(a) for a in sdf]
        g.step(1)                      # a pending projection, as before every replay
    o.step(1)
    s.synchronize()
    hip = ctypes.CDLL("libamdhip64.so")
    graph, gexec = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipStreamBeginCapture(ctypes.c_void_p(s.cuda_stream), 1) == 0
    try:
        g.set_geometry(*bufs)
        g.step(1)
    finally:
        rc = hip.hipStreamEndCapture(ctypes.c_void_p(s.cuda_stream), ctypes.byref(graph))
    assert rc == 0 and graph.value
    assert hip.hipGraphInstantiate(ctypes.byref(gexec), graph, None, None, ctypes.c_size_t(0)) == 0
    try:
        for n in range(3):
            centre = centre + np.array(vel) * c.dt
            sdf = _body_sdf(c, centre, 0.3)
            o.set_geometry(*sdf)
            o.step(1)
            with torch.cuda.stream(s):
                for b, a in zip(bufs, sdf):
                    b.copy_(torch.from_numpy(a))
            assert hip.hipGraphLaunch(gexec, ctypes.c_void_p(s.cuda_stream)) == 0
            s.synchronize()
            with torch.cuda.stream(s):
                errs, _ = _errs(g, o)
            _say(f"caller graph, replay {n + 1}: {['%.1e' % e for e in errs]}")
            assert max(errs) < 1e-12
    finally:
        hip.hipGraphExecDestroy(gexec)
        hip.hipGraphDestroy(graph)
    g.close()


def test_geometry_beyond_the_list_capacity():
    """A geometry with more immersed-boundary points than the lists reserved at the first
    one is reported by ibm_stats (IBM_ERR_STATE); giving it again resizes the lists, and
    the step then equals the oracle's."""
    from paper_2506_14328_amd.ibm import IBM_ERR_STATE, IbmError
    c = I.Case(nx=32, ny=33, nz=16, lx=2.0, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=0.02, dt=0.01, q_target_or_pi=1.0,
               seed=9, geometry="flat", geo_params=(0.0,))

    def body(r):
        def fn(X, Y, Z):
            dx = X - 1.0
            dx -= c.lx * np.round(dx / c.lx)
            dz = Z - 0.5
            dz -= c.lz * np.round(dz / c.lz)
            return np.minimum(np.sqrt(dx * dx + Y * Y + dz * dz) - r, 1.0 - np.abs(Y))
        return I._sample(c, fn)

    small, big = body(0.05), body(0.8)
    u0, v0, w0 = I.laminar_plus_solenoidal(c, big, c.seed, amp=0.05)
    st = (u0, v0, w0, np.zeros_like(u0))
    g = gpu_grid(c, small, st)
    n_small = g.stats()["n_ibm"]
    g.set_geometry(*[to_dev(a) for a in big])
    with pytest.raises(IbmError) as e:
        g.stats()
    assert e.value.code == IBM_ERR_STATE
    g.set_geometry(*[to_dev(a) for a in big])      # resized now
    g.set_state(*[to_dev(a) for a in st])
    o = Oracle(OGrid.from_case(c))
    o.set_geometry(*big)
    o.set_state(*st)
    g.step(2)
    o.step(2)
    errs, _ = _errs(g, o)
    s = g.stats()
    _say(f"capacity: first geometry {n_small}, larger {s['n_ibm']}; after resizing {['%.1e' % x for x in errs]}")
    assert s["n_ibm"] == [int((o.lam[k] > 0).sum()) for k in "uvw"]
    assert max(errs) < 1e-12
    g.close()
