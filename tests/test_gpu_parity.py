"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: binning and pair counts bit-exact; single-evaluation forces max-abs
<= 1e-4 in mixed precision (FP32 forces, a = 25 scale) and <= 1e-9 in FP64;
10-step trajectories <= 1e-3 (mixed) and <= 1e-9 (FP64); long-run kT and p
within 1% of the oracle's.
"""
import numpy as np
import pytest

import oracle
from paper_1804_06205_amd import dpd
from paper_1804_06205_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_F = {"mixed": 1e-4, "fp64": 1e-9}
TOL_X10 = {"mixed": 1e-3, "fp64": 1e-9}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dpd.lib()
    oracle.lib()


def _min_image_diff(a, b, L):
    d = np.asarray(a) - np.asarray(b)
    L = np.asarray(L, dtype=float)
    return d - L * np.rint(d / L)


def _gpu_force(w, precision, s=0):
    """GPU force F(x, v; s) of the workload's state (vt = v)."""
    with dpd.System.from_workload(w, precision=precision) as g:
        g.set_state(w.pos, w.vel, None, s)
        _, _, f, _ = g.get_state()
    return f


def _oracle_force(w, s=0):
    return oracle.forces(w.pos, w.vel, w.L, w.types, w.params(), w.seed, s, w.bonds())


# --------------------------------------------------------------------------
# Binning and pair counts: bit-exact.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("L", [3.0, 5.0, 10.0, 7.5])
def test_binning_matches_oracle_bit_exact(L):
    w = W.fluid(L, seed=int(L * 10) + 1)
    pos = w.pos.copy()
    rng = np.random.default_rng(5)
    idx = rng.choice(w.n, size=w.n // 8, replace=False)
    h = L / np.floor(L)
    pos[idx, 0] = np.floor(pos[idx, 0] / h) * h            # exactly on cell faces
    pos[idx[: len(idx) // 2], 1] = np.nextafter(L, 0.0)    # just below L
    w.pos = pos
    with dpd.System.from_workload(w) as g:
        cell, count = g.get_cells()
    cxyz, ocount, _, _ = oracle.bin_cells(pos, w.L)
    nx = int(np.floor(L))
    lin = (cxyz[:, 2] * nx + cxyz[:, 1]) * nx + cxyz[:, 0]
    np.testing.assert_array_equal(cell, lin)
    np.testing.assert_array_equal(count, ocount)


def _cells_vs_oracle(g, x, L):
    """The system's current cell list against the oracle's binning of the
    system's own positions x: per-particle cells and counts, bit-exact."""
    cell, count = g.get_cells()
    cxyz, ocount, _, _ = oracle.bin_cells(x, L)
    nc = np.floor(np.asarray(L, dtype=float)).astype(np.int64)
    np.testing.assert_array_equal(cell, (cxyz[:, 2] * nc[1] + cxyz[:, 1]) * nc[0] + cxyz[:, 0])
    np.testing.assert_array_equal(count, ocount)


@pytest.mark.parametrize("case,steps,precision", [
    ("fluid_L96", 5, "mixed"),             # unit cells: the divide-free binning
    ("fluid_L7.5", 5, "mixed"),            # cell edge 7.5/7: the FP64 divide
    ("fluid_L7.5", 5, "fp64"),
    ("fluid_6x7.5x8", 6, "mixed"),         # non-cubic cells
    ("peptide_L10", 7, "mixed"),
])
def test_binning_inside_steps_matches_oracle_bit_exact(case, steps, precision):
    # After fused step passes, the cell list the kernels built (integrate-1 and
    # the append into the next layout) equals the oracle's binning of the
    # positions those passes produced.  steps = 1 goes through the begin pass
    # only; more steps end with a list built by a fused pass.
    w = {"fluid_L96": lambda: W.cfg_fluid_L96(),
         "fluid_L7.5": lambda: W.fluid(7.5, seed=3),
         "fluid_6x7.5x8": lambda: W.fluid((6.0, 7.5, 8.0), seed=9),
         "peptide_L10": lambda: W.peptide(10.0, seed=10, nchains=8, nbeads=20)}[case]()
    with dpd.System.from_workload(w, precision=precision) as g:
        for k in (1, steps - 1):
            g.step(k)
            x, _, _, t = g.get_state(force=False)
            _cells_vs_oracle(g, x, w.L)
        assert t == steps


def test_binning_of_exact_face_positions_inside_steps():
    # No forces (a = gamma = sigma = 0), dt = 1/16, positions on a 2^-8 grid
    # and velocities m/16: every drift dt v is exact, so particles move on the
    # grid and land exactly on cell faces (and on 0 after wrapping from L)
    # every step.  The kernels' positions equal the exact ballistic ones and
    # their cells equal the oracle's, bit for bit, at every step.
    L = 10.0
    rng = np.random.default_rng(77)
    n = 3000
    pos = rng.integers(0, 256 * 10, size=(n, 3)).astype(np.float64) / 256.0
    vel = rng.integers(-16, 17, size=(n, 3)).astype(np.float64) / 16.0
    dt = 1.0 / 16.0
    for precision in ("mixed", "fp64"):
        with dpd.System([L] * 3, pos, vel, precision=precision) as g:
            g.set_params([[0.0]], 0.0, 0.0, 1.0, dt, 0.65)
            x = pos.copy()
            faces = 0
            for k in range(12):
                g.step(1 if k % 2 == 0 else 3)
                for _ in range(1 if k % 2 == 0 else 3):
                    x = np.mod(x + dt * vel, L)
                xg, vg, _, _ = g.get_state(force=False)
                np.testing.assert_array_equal(xg, x)
                np.testing.assert_array_equal(vg, vel)
                faces += int((xg == np.floor(xg)).sum())
                _cells_vs_oracle(g, xg, [L] * 3)
        # About 3n / 256 = 35 coordinates sit exactly on a face per check.
        assert faces > 200, (precision, faces)


def test_non_cubic_box_binning():
    rng = np.random.default_rng(3)
    L = np.array([3.0, 4.5, 7.25])
    n = int(3 * L.prod())
    pos = rng.uniform(0, 1, (n, 3)) * L
    vel = rng.normal(size=(n, 3))
    with dpd.System(L, pos, vel) as g:
        cell, count = g.get_cells()
    cxyz, ocount, _, _ = oracle.bin_cells(pos, L)
    nc = np.floor(L).astype(int)
    np.testing.assert_array_equal(cell, (cxyz[:, 2] * nc[1] + cxyz[:, 1]) * nc[0] + cxyz[:, 0])
    np.testing.assert_array_equal(count, ocount)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_pair_count_exact_on_quantized_positions(precision):
    w = W.fluid(10.0, seed=7, quantize=8)
    with dpd.System.from_workload(w, precision=precision) as g:
        o = g.observables()
    ref = oracle.observables(w.pos, w.vel, w.L, w.types, w.a)
    assert o["npairs"] == ref["npairs"]


# --------------------------------------------------------------------------
# Single force evaluations.
# --------------------------------------------------------------------------

def _binary_fluid(L, seed):
    # Two particle types and no bonds: the step kernel built without the bond
    # code, with the a_ij table (a_AA = a_BB = 25, a_AB = 40).
    w = W.fluid(L, seed=seed, name=f"binary_L{L:g}")
    w.types = (np.arange(w.n) % 2).astype(np.uint8)
    w.ntypes = 2
    w.a = np.array([[25.0, 40.0], [40.0, 25.0]])
    return w


def _cases():
    return {
        "fluid_L10": W.fluid(10.0, seed=1),
        "fluid_L3": W.fluid(3.0, seed=2),
        "fluid_L7.5": W.fluid(7.5, seed=3),
        "binary_L8": _binary_fluid(8.0, 9),
        "melt_L8": W.melt(8.0, seed=4),
        "peptide_L8": W.peptide(8.0, seed=5, nchains=6, nbeads=20),
        "helix_L6": W.helix(6.0, seed=6, beads=12),
        # Non-cubic cells (edges 1, 7.5/7, 1): the kernels' offsets frame
        # with explicit whole-cell shifts, in both precisions.
        "fluid_6x7.5x8": W.fluid((6.0, 7.5, 8.0), seed=7),
        "peptide_6x7.5x8": W.peptide((6.0, 7.5, 8.0), seed=8, nchains=4, nbeads=20),
    }


@pytest.mark.parametrize("name", list(_cases()))
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_force_parity(name, precision):
    w = _cases()[name]
    for s in (0, 17):
        fg = _gpu_force(w, precision, s)
        fo = _oracle_force(w, s)
        err = np.abs(fg - fo).max()
        print(f"{name} {precision} s={s}: force max-abs {err:.3e}")
        assert err <= TOL_F[precision], (name, s, err)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_force_parity_thermalised_state(precision):
    # A state taken from a trajectory (not a uniform random start).
    w = W.peptide(8.0, seed=9, nchains=4, nbeads=20)
    st = oracle.State.from_workload(w).step(30)
    w.pos, w.vel = st.pos, st.vel
    err = np.abs(_gpu_force(w, precision, 30) - _oracle_force(w, 30)).max()
    assert err <= TOL_F[precision]


@pytest.mark.parametrize("n", [2, 3, 9])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_nearly_empty_box(n, precision):
    # Almost every cell and most bricks hold nothing; n = 2 is the smallest
    # system the boundary accepts.  Particles are placed in pairs within the
    # cutoff so there are forces to compare.
    w = W.fluid(7.0, seed=50 + n, precision=precision)
    rng = np.random.default_rng(n)
    pos = rng.uniform(0, 7.0, (n, 3))
    pos[1::2] = (pos[0:n - 1:2] + rng.uniform(-0.4, 0.4, (n // 2, 3))) % 7.0
    w.pos, w.vel, w.types = pos, w.vel[:n].copy(), w.types[:n].copy()
    fo = _oracle_force(w, 5)
    assert np.abs(fo).max() > 0
    err = np.abs(_gpu_force(w, precision, 5) - fo).max()
    with dpd.System.from_workload(w, precision=precision) as g:
        g.step(10)
        xg, _, _, _ = g.get_state()
    st = oracle.State.from_workload(w).step(10)
    dx = np.abs(_min_image_diff(xg, st.pos, w.L)).max()
    print(f"n={n} {precision}: force max-abs {err:.3e}, 10-step position {dx:.3e}", flush=True)
    assert err <= TOL_F[precision]
    assert dx <= TOL_X10[precision]


def test_momentum_conservation():
    w = W.peptide(8.0, seed=12, nchains=6, nbeads=20)
    f = _gpu_force(w, "mixed", 3)
    assert np.abs(f.sum(0)).max() <= 1e-5 * np.sqrt(w.n) * np.abs(f).max()
    f64 = _gpu_force(w, "fp64", 3)
    assert np.abs(f64.sum(0)).max() <= 1e-10 * np.abs(f64).max()


# --------------------------------------------------------------------------
# Trajectories.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["fluid_L10", "binary_L8", "melt_L8", "peptide_L8", "helix_L6",
                                  "fluid_6x7.5x8", "peptide_6x7.5x8"])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_ten_step_trajectory(name, precision):
    w = _cases()[name]
    with dpd.System.from_workload(w, precision=precision) as g:
        g.step(10)
        xg, vg, fg, step = g.get_state()
    assert step == 10
    st = oracle.State.from_workload(w).step(10)
    dx = np.abs(_min_image_diff(xg, st.pos, w.L)).max()
    assert dx <= TOL_X10[precision], dx


def test_step_splitting_and_determinism_are_bitwise():
    w = W.peptide(8.0, seed=21, nchains=4, nbeads=20)
    runs = []
    for split in ((7,), (3, 4), (1, 1, 5)):
        with dpd.System.from_workload(w) as g:
            for k in split:
                g.step(k)
            runs.append(g.get_state())
    for r in runs[1:]:
        for a, b in zip(r[:3], runs[0][:3]):
            np.testing.assert_array_equal(a, b)


def test_checkpoint_resume_is_bitwise():
    w = W.melt(8.0, seed=22)
    with dpd.System.from_workload(w) as g:
        g.step(20)
        ref = g.get_state()
    with dpd.System.from_workload(w) as g:
        g.step(8)
        x, v, f, s = g.get_state()
    with dpd.System.from_workload(w) as g2:
        g2.set_state(x, v, f, s)
        g2.step(12)
        got = g2.get_state()
    for a, b in zip(got[:3], ref[:3]):
        np.testing.assert_array_equal(a, b)
    assert got[3] == 20


# --------------------------------------------------------------------------
# Observables.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_observables_match_oracle_on_same_state(precision):
    w = W.peptide(8.0, seed=31, nchains=6, nbeads=20)
    with dpd.System.from_workload(w, precision=precision) as g:
        g.step(5)
        o = g.observables()
        x, v, _, _ = g.get_state(force=False)
    ref = oracle.observables(x, v, w.L, w.types, w.a, w.bonds())
    rt = 1e-5 if precision == "mixed" else 1e-10
    for k in ("ke", "u_pair", "u_bond", "w_pair", "w_bond", "pressure", "kT"):
        assert abs(o[k] - ref[k]) <= rt * max(1.0, abs(ref[k])), (k, o[k], ref[k])
    np.testing.assert_allclose(o["momentum"], [ref["px"], ref["py"], ref["pz"]], atol=1e-6)
    assert abs(o["npairs"] - ref["npairs"]) <= (2 if precision == "mixed" else 0)


# --------------------------------------------------------------------------
# Full-size workload (fluid L = 96, 2,654,208 particles).
# --------------------------------------------------------------------------

def test_full_size_observables_match_oracle():
    # The observables pass and the deterministic reductions over 2.65M tags,
    # on the GPU's own state after three fused steps on the bench's brick.
    # The oracle tests r < 1 on the FP64 positions, the kernel on their 2^-29
    # fixed-point offsets: pairs within ~2e-9 of the cutoff (about 0.2 per
    # evaluation here) may be counted on one side only.
    w = W.cfg_fluid_L96()
    with dpd.System.from_workload(w) as g:
        g.set_variant(1)
        g.step(3)
        o = g.observables()
        x, v, _, _ = g.get_state(force=False)
    ref = oracle.observables(x, v, w.L, w.types, w.a, w.bonds())
    for k in ("ke", "u_pair", "w_pair", "pressure", "kT"):
        assert abs(o[k] - ref[k]) <= 1e-5 * max(1.0, abs(ref[k])), (k, o[k], ref[k])
    np.testing.assert_allclose(o["momentum"], [ref["px"], ref["py"], ref["pz"]], atol=1e-6)
    assert abs(o["npairs"] - ref["npairs"]) <= 4, (o["npairs"], ref["npairs"])


def test_full_size_fluid_binning_and_forces():
    w = W.cfg_fluid_L96()
    with dpd.System.from_workload(w) as g:
        cell, count = g.get_cells()
        g.set_state(w.pos, w.vel, None, 0)
        _, _, fg, _ = g.get_state()
    cxyz, ocount, _, _ = oracle.bin_cells(w.pos, w.L)
    np.testing.assert_array_equal(cell, (cxyz[:, 2] * 96 + cxyz[:, 1]) * 96 + cxyz[:, 0])
    np.testing.assert_array_equal(count, ocount)
    fo = _oracle_force(w, 0)
    err = np.abs(fg - fo).max()
    print(f"fluid_L96 force max-abs {err:.3e}")
    assert err <= TOL_F["mixed"], err


def test_full_size_fused_steps_on_the_bench_brick():
    # The bench's launch configuration: the 5x4x4 brick, fused step passes,
    # the full 2.65M-particle box; ten steps against the oracle's.
    w = W.cfg_fluid_L96()
    with dpd.System.from_workload(w) as g:
        g.set_variant(1)
        assert dpd.variants()[1][:3] == (5, 4, 4)
        g.step(10)
        xg, vg, fg, t = g.get_state()
    st = oracle.State.from_workload(w)
    st.step(10)
    dx = np.abs(_min_image_diff(xg, st.pos, w.L)).max()
    dv = np.abs(vg - st.vel).max()
    df = np.abs(fg - st.force).max()
    print(f"fluid_L96 10 fused steps vs oracle: pos {dx:.3e} vel {dv:.3e} force {df:.3e}; "
          f"momentum {np.abs(vg.sum(axis=0)).max():.3e}")
    assert t == 10
    assert dx <= TOL_X10["mixed"]
    # The 1e-4 force bar is for one evaluation on identical inputs (the test
    # above).  After ten steps the two trajectories differ by ~3e-6 in
    # position, and the closest of 2.65M pairs (~0.004 apart) turn that into
    # force differences of ~3e-4 (observed): chaos, not a kernel error.
    # Velocities stay close (observed 2.2e-5).
    assert dv <= 1e-3 and df <= 1e-2
    assert np.abs(vg.sum(axis=0)).max() <= 1e-5 * np.sqrt(w.n) * np.abs(vg).max()


@pytest.mark.parametrize("cfg", ["melt_L32", "peptide_L40"])
def test_full_size_bonded_configurations(cfg):
    # The bonded configurations at their full sizes (98 304 and 192 000
    # particles; harmonic bonds, and 1-3 / 1-5 standard Morse terms in the
    # peptide): forces of the initial state, then ten fused steps on the
    # 5x4x4 brick, against the oracle.
    w = {"melt_L32": W.cfg_melt_L32, "peptide_L40": W.cfg_peptide_L40}[cfg]()
    fo = _oracle_force(w, 0)
    with dpd.System.from_workload(w) as g:
        g.set_variant(1)
        g.set_state(w.pos, w.vel, None, 0)
        _, _, fg, _ = g.get_state()
        g.step(10)
        xg, vg, _, t = g.get_state()
    err = np.abs(fg - fo).max()
    st = oracle.State.from_workload(w)
    st.step(10)
    dx = np.abs(_min_image_diff(xg, st.pos, w.L)).max()
    dv = np.abs(vg - st.vel).max()
    print(f"{cfg} (n={w.n}): force max-abs {err:.3e}; 10 steps pos {dx:.3e} vel {dv:.3e}")
    assert err <= TOL_F["mixed"]
    assert t == 10 and dx <= TOL_X10["mixed"] and dv <= 1e-2


@pytest.mark.parametrize("chains", [False, True])
def test_paper_sweep_box(chains):
    # The paper's N = 50 000 benchmark box (L = 25.54: 25 cells of edge
    # 1.0217 per axis, so the integer brick frame with non-unit cells), as the
    # plain fluid (Table 1) and with the Table 3 chains (25 chains of the
    # alpha-helix deck's 1-2 / 1-3 harmonic and 1-3 / 1-5 modified Morse
    # records, dt = 0.02): forces of the initial state, then ten steps, and
    # the cell list the last step built.
    w = W.sweep_box(50000, chains=chains)
    assert abs(w.L[0] - 25.544) < 1e-3 and w.n == 50000
    fo = _oracle_force(w, 0)
    with dpd.System.from_workload(w) as g:
        assert g.info()["nx"] == 25
        g.set_state(w.pos, w.vel, None, 0)
        _, _, fg, _ = g.get_state()
        g.step(10)
        xg, vg, _, t = g.get_state()
        _cells_vs_oracle(g, xg, w.L)
    err = np.abs(fg - fo).max()
    st = oracle.State.from_workload(w)
    st.step(10)
    dx = np.abs(_min_image_diff(xg, st.pos, w.L)).max()
    print(f"sweep N=50000 chains={chains}: force max-abs {err:.3e}; 10 steps pos {dx:.3e}",
          flush=True)
    assert err <= TOL_F["mixed"]
    assert t == 10 and dx <= TOL_X10["mixed"]


def test_coincident_particles():
    # Two particles exactly on top of each other: no force between them (e is
    # undefined; Eq. 4 needs r > 0), the rest as the oracle has it; the pair
    # count includes them.
    w = W.fluid(5.0, seed=12)
    w.pos[1] = w.pos[0]
    for prec in ("mixed", "fp64"):
        with dpd.System.from_workload(w, precision=prec) as g:
            g.set_state(w.pos, w.vel, None, 0)
            _, _, fg, _ = g.get_state()
            o = g.observables()
        fo = _oracle_force(w, 0)
        assert np.all(np.isfinite(fg))
        assert np.abs(fg - fo).max() <= TOL_F[prec]
        ref = oracle.observables(w.pos, w.vel, w.L, w.types, w.a)
        assert o["npairs"] == ref["npairs"]


def test_full_size_pair_count_quantized():
    w = W.fluid(96.0, seed=3, quantize=8)
    with dpd.System.from_workload(w) as g:
        o = g.observables()
    _, _, _, n_or = oracle.pair_forces(w.pos, w.vel, w.L, w.a, 0.0, 0.0, 1.0, 0, 0)
    assert o["npairs"] == n_or


# --------------------------------------------------------------------------
# Long-run statistics (fluid L = 10, FP64, as the small benchmark workload).
# --------------------------------------------------------------------------

def test_long_run_temperature_and_pressure():
    w = W.cfg_fluid_L10()
    g = dpd.System.from_workload(w)
    st = oracle.State.from_workload(w)
    g.step(200)
    st.step(200)
    tg, pg, to, po = [], [], [], []
    for _ in range(200):
        g.step(5)
        st.step(5)
        og = g.observables()
        oo = st.observables()
        tg.append(og["kT"])
        pg.append(og["pressure"])
        to.append(oo["kT"])
        po.append(oo["pressure"])
    g.close()
    assert abs(np.mean(tg) - np.mean(to)) <= 0.01 * np.mean(to)
    assert abs(np.mean(pg) - np.mean(po)) <= 0.01 * np.mean(po)


def test_long_run_temperature_and_pressure_mixed_precision():
    # The mixed path (FP32 forces and velocities, hardware log/cos/rsqrt in the
    # pair term) over a long run: peptide-like chains in solvent at L = 12
    # (11 chains of 20, the peptide workload's 4% chain fraction), the
    # standard 1-3 and 1-5 Morse terms at dt = 0.04, 2000 steps.  Time averages
    # of kT and p after 200 steps agree with the oracle's within 1%, and the
    # run stays stable (the stiff Morse at this dt).
    w = W.peptide(12.0, seed=44, nchains=11, nbeads=20)
    assert w.precision == "mixed"
    g = dpd.System.from_workload(w)
    st = oracle.State.from_workload(w)
    g.step(200)
    st.step(200)
    tg, pg, to, po = [], [], [], []
    for _ in range(360):
        g.step(5)
        st.step(5)
        og = g.observables()
        oo = st.observables()
        tg.append(og["kT"])
        pg.append(og["pressure"])
        to.append(oo["kT"])
        po.append(oo["pressure"])
    xg, _, _, t = g.get_state(force=False)
    g.close()
    print(f"mixed long run: kT {np.mean(tg):.4f} vs {np.mean(to):.4f}, "
          f"p {np.mean(pg):.3f} vs {np.mean(po):.3f}", flush=True)
    assert t == 2000 and np.all(np.isfinite(xg))
    assert abs(np.mean(tg) - np.mean(to)) <= 0.01 * np.mean(to)
    assert abs(np.mean(pg) - np.mean(po)) <= 0.01 * np.mean(po)


# --------------------------------------------------------------------------
# The 32-bit step counter.
# --------------------------------------------------------------------------

def test_step_counter_limit():
    # The step index keys the noise as a 32-bit word; the library runs up to
    # 2^32 - 1 and refuses to pass it.  Near the limit the trajectory still
    # follows the oracle and the cell list is the one of the current state.
    w = W.peptide(6.0, seed=60, nchains=2, nbeads=12)
    top = 2 ** 32 - 1
    with dpd.System.from_workload(w) as g:
        with pytest.raises(dpd.DPDError) as e:
            g.set_state(w.pos, w.vel, None, top + 1)
        assert e.value.code == dpd.EINVAL
        g.set_state(w.pos, w.vel, None, top - 4)
        g.step(4)
        with pytest.raises(dpd.DPDError) as e:
            g.step(1)
        assert e.value.code == dpd.EINVAL
        g.step(0)
        x, v, f, t = g.get_state()
        assert t == top
        _cells_vs_oracle(g, x, w.L)
    st = oracle.State(w.pos, w.vel, w.L, w.types, w.params(), w.seed, w.bonds(),
                      step=top - 4).step(4)
    assert np.abs(_min_image_diff(x, st.pos, w.L)).max() <= TOL_X10["mixed"]
    assert np.abs(f - st.force).max() <= TOL_F["mixed"]


# --------------------------------------------------------------------------
# Error handling (host-forced; every kernel exits normally).
# --------------------------------------------------------------------------

def test_cell_capacity_overflow_is_reported():
    w = W.fluid(5.0, seed=40)
    pos = w.pos.copy()
    pos[:20] = [1.5, 1.5, 1.5] + 0.01 * np.arange(20)[:, None]   # 20 in one cell
    with pytest.raises(dpd.DPDError) as e:
        dpd.System(w.L, pos, w.vel, cell_capacity=8)
    assert e.value.code == dpd.ECAPACITY


def test_argument_errors():
    w = W.fluid(5.0, seed=41)
    with pytest.raises(dpd.DPDError) as e:
        dpd.System([2.5, 5, 5], w.pos, w.vel)
    assert e.value.code == dpd.EBOX
    with dpd.System.from_workload(w) as g:
        with pytest.raises(dpd.DPDError) as e:
            g.add_bonds([1], [0], [0], [0.0], [1.0], [0.0])
        assert e.value.code == dpd.ERANGE
        with pytest.raises(dpd.DPDError) as e:
            g.set_params([[25.0]], 4.5, 3.0, 1.0, -0.04)
        assert e.value.code == dpd.EINVAL
        g.step(1)
        with pytest.raises(dpd.DPDError) as e:
            g.set_params([[25.0]], 4.5, 3.0, 1.0, 0.04)
        assert e.value.code == dpd.ESTATE


def test_nonfinite_state_is_rejected():
    w = W.fluid(5.0, seed=42)
    with dpd.System.from_workload(w) as g:
        v = w.vel.copy()
        v[3, 1] = np.nan
        with pytest.raises(dpd.DPDError) as e:
            g.set_state(w.pos, v)
        assert e.value.code == dpd.EINVAL


# --------------------------------------------------------------------------
# Brick variants, chunked neighbourhoods and the autotuner.
# --------------------------------------------------------------------------

def test_dense_box_uses_chunked_neighbourhoods():
    # rho = 6: a 2x2x2 brick's 64-cell neighbourhood holds ~384 particles,
    # more than its 320-slot tile, so the kernel processes it in chunks.
    w = W.fluid(6.0, rho=6.0, seed=50)
    with dpd.System.from_workload(w) as g:
        g.set_variant(4)
        g.set_state(w.pos, w.vel, None, 2)
        _, _, f, _ = g.get_state()
        g.step(3)
        x, _, _, _ = g.get_state()
    fo = _oracle_force(w, 2)
    assert np.abs(f - fo).max() <= TOL_F["mixed"]
    st = oracle.State(w.pos, w.vel, w.L, w.types, w.params(), w.seed, step=2).step(3)
    assert np.abs(_min_image_diff(x, st.pos, w.L)).max() <= TOL_X10["mixed"]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("system", ["peptide", "melt", "sweep_chains", "binary"])
def test_every_brick_variant_gives_bitwise_identical_steps(precision, system):
    # The bond terms are scheduled per wave: dealt one per lane where a few
    # lanes own several records (peptide chains in solvent), each lane's own
    # records four at a time where bonds are spread over the lanes or more
    # than 64 (the melt); Table 3's box has waves of both kinds.  Different
    # bricks put different particles in a wave, so the same particle meets
    # either schedule, and the sums must agree to the bit.
    w = {"peptide": lambda: W.peptide(10.0, seed=51, nchains=5, nbeads=20),
         "melt": lambda: W.melt(8.0, seed=52),
         "sweep_chains": lambda: W.sweep_box(5000, chains=True),
         "binary": lambda: _binary_fluid(10.0, 54)}[system]()
    ref = None
    for v in range(len(dpd.variants())):
        with dpd.System.from_workload(w, precision=precision) as g:
            g.set_variant(v)
            g.step(6)
            got = g.get_state()
        if ref is None:
            ref = got
        else:
            for a, b in zip(got[:3], ref[:3]):
                np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("rho", [4.5, 6.0])
def test_chunked_neighbourhoods_give_bitwise_identical_steps(rho):
    # At rho = 4.5 the small bricks' neighbourhoods mostly fit their tiles
    # while the large ones are split into chunks; at rho = 6 every variant
    # splits, at different cell boundaries.  Each particle still adds its
    # pairs in the same order, so every variant gives the same bits.
    w = W.fluid(8.0, rho=rho, seed=53)
    ref = None
    for v in range(len(dpd.variants())):
        with dpd.System.from_workload(w) as g:
            g.set_variant(v)
            g.step(4)
            got = g.get_state()
        if ref is None:
            ref = got
        else:
            for a, b in zip(got[:3], ref[:3]):
                np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_large_cell_capacity_gives_bitwise_identical_steps(precision):
    # With 1024 slots per cell a brick's halo counts may add up to 2^16 or
    # more, so the brick prologue takes its wide prefix scan instead of the
    # packed one; the layout is padded differently, which the tag-order
    # staging hides: every combination gives the same bits.
    w = W.peptide(10.0, seed=51, nchains=5, nbeads=20)
    got = {}
    for cap in (0, 1024):
        for v in (1, 4):
            with dpd.System.from_workload(w, precision=precision, cell_capacity=cap) as g:
                g.set_variant(v)
                g.step(6)
                got[cap, v] = g.get_state()
    ref = got[0, 1]
    for key, st in got.items():
        for a, b in zip(st[:3], ref[:3]):
            np.testing.assert_array_equal(a, b, err_msg=str(key))


def test_autotune_leaves_the_state_unchanged():
    w = W.melt(12.0, seed=52)
    with dpd.System.from_workload(w) as g:
        g.step(4)
        before = g.get_state()
        v, ms = g.autotune(2)
        assert 0 <= v < len(dpd.variants()) and ms > 0
        after = g.get_state()
        for a, b in zip(after[:3], before[:3]):
            np.testing.assert_array_equal(a, b)
    with dpd.System.from_workload(w) as g2:
        g2.step(7)
        ref = g2.get_state()
    with dpd.System.from_workload(w) as g3:
        g3.step(4)
        g3.autotune(2)
        g3.step(3)
        got = g3.get_state()
    for a, b in zip(got[:3], ref[:3]):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_device_pair_noise_matches_oracle(precision):
    # The kernels' Philox4x32-10 + Box-Muller against the oracle's independent
    # implementation: FP32 agrees to its rounding of theta (|theta| <= 5.8),
    # FP64 to ~1e-13.
    rng = np.random.default_rng(8)
    m = 200_000
    ti = rng.integers(0, 2 ** 32, size=m, dtype=np.uint64).astype(np.uint32)
    tj = rng.integers(0, 2 ** 32, size=m, dtype=np.uint64).astype(np.uint32)
    s = rng.integers(0, 2 ** 32, size=m, dtype=np.uint64).astype(np.uint32)
    seed = 0x0123456789ABCDEF
    got = dpd.pair_noise(seed, ti, tj, s, precision)
    ref = oracle.pair_noise_batch(seed, ti, tj, s)
    tol = 1.5e-6 if precision == "mixed" else 1e-12
    assert np.abs(got - ref).max() <= tol
    np.testing.assert_array_equal(dpd.pair_noise(seed, tj, ti, s, precision), got)
