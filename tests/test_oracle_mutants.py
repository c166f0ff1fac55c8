"""The oracle's pins are strong enough to catch plausible mistakes.

Each case below plants one mistake in a copy of ``oracle/tvd_oracle.c`` (a
dropped term, a wrong sign, a shifted index, a transposed operand, the wrong
state in the full step, a wrong region rule, a misplaced boundary flux), builds it with gcc into a
temporary directory and runs the pins of ``test_oracle_pins.py`` against it
in a child process.  At least one pin must fail for every mistake.  The
planted copies live only in the temporary directory; the real oracle is
never modified.
"""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

MUTANTS = {
    "pressure dropped from the normal momentum flux":
        ("F[1 + d] = m_d * v_d + P;", "F[1 + d] = m_d * v_d;"),
    "pressure dropped from the energy flux":
        ("F[4] = (e + P) * v_d;", "F[4] = e * v_d;"),
    "left-moving flux with the wrong sign":
        ("FL[k] = 0.5 * (c * u[k] - F[k]);", "FL[k] = 0.5 * (c * u[k] + F[k]);"),
    "freezing speed without |v|":
        ("const double c = fabs(v_d) + cs;", "const double c = cs;"),
    "sound speed without gamma":
        ("const double cs = sqrt(gamma * P / rho);\n    const double c = fabs(v_d) + cs;",
         "const double cs = sqrt(P / rho);\n    const double c = fabs(v_d) + cs;"),
    "kinetic energy without the 1/2":
        ("const double kin = 0.5 * (m_d * v_d", "const double kin = 1.0 * (m_d * v_d"),
    "transverse momentum advected by its own velocity":
        ("F[1 + t1] = m_t1 * v_d;", "F[1 + t1] = m_t1 * v_t1;"),
    "half step over the full dt":
        ("/ dh * (dt / 2.0);", "/ dh * dt;"),
    "half step with the flux difference reversed":
        ("(G[j * NVAR + k] - G[(j - 1) * NVAR + k])", "(G[(j - 1) * NVAR + k] - G[j * NVAR + k])"),
    "full step taken from the midpoint state":
        ("out[i * NVAR + k] = q[j * NVAR + k] -", "out[i * NVAR + k] = h[j * NVAR + k] -"),
    "right-moving limiter reads the wrong cells":
        ("const double dR1 = (FRh[j * NVAR + k] - FRh[(j - 1) * NVAR + k]) / 2.0;",
         "const double dR1 = (FRh[(j + 1) * NVAR + k] - FRh[j * NVAR + k]) / 2.0;"),
    "left-moving flux upwinded from the wrong cell":
        ("const double Lf = FLh[(j + 1) * NVAR + k] + oracle_vanleer(dL1, dL2);",
         "const double Lf = FLh[j * NVAR + k] + oracle_vanleer(dL1, dL2);"),
    "arithmetic-mean limiter":
        ("if (dF1 * dF2 > 0.0) return 2.0 * dF1 * dF2 / (dF1 + dF2);",
         "if (dF1 * dF2 > 0.0) return 0.5 * (dF1 + dF2);"),
    "limiter active at extrema":
        ("if (dF1 * dF2 > 0.0) return", "if (dF1 + dF2 != 0.0) return"),
    "region rule drops the ghosts of later axes":
        ("lo[a] = later ? -GHOST : 0;", "lo[a] = 0;"),
    "backward triple sweeps in forward order":
        ("bwd[3] = {2, 1, 0};", "bwd[3] = {0, 1, 2};"),
    "signal speed uses the sum of the velocities":
        ("const double s = cs + vmax;", "const double s = cs + fabs(vx) + fabs(vy) + fabs(vz);"),
    "boundary flux taken one interface off":
        ("hface[i * NVAR + k] = H[(i + GHOST - 1) * NVAR + k];",
         "hface[i * NVAR + k] = H[(i + GHOST) * NVAR + k];"),
    "boundary flux face coordinates transposed":
        ("const int a = a1 > a2 ? p1 : p2;\n                    const int b = a1 > a2 ? p2 : p1;",
         "const int a = a1 > a2 ? p2 : p1;\n                    const int b = a1 > a2 ? p1 : p2;"),
    "freezing speed taken at time t in the midpoint fluxes":
        ("""        oracle_split_fluxes(h + j * NVAR, d, gamma, p_floor, FRh + j * NVAR,
                            FLh + j * NVAR, cnt);""",
         """    {
        const double ct = oracle_split_fluxes(q + j * NVAR, d, gamma, p_floor, FRh + j * NVAR,
                                              FLh + j * NVAR, NULL);
        const double ch = oracle_split_fluxes(h + j * NVAR, d, gamma, p_floor, FRh + j * NVAR,
                                              FLh + j * NVAR, cnt);
        for (int k = 0; k < NVAR; ++k) {
            FRh[j * NVAR + k] += 0.5 * (ct - ch) * h[j * NVAR + k];
            FLh[j * NVAR + k] += 0.5 * (ct - ch) * h[j * NVAR + k];
        }
    }"""),
    "limiter on unhalved differences":
        ("""            const double dR1 = (FRh[j * NVAR + k] - FRh[(j - 1) * NVAR + k]) / 2.0;
            const double dR2 = (FRh[(j + 1) * NVAR + k] - FRh[j * NVAR + k]) / 2.0;""",
         """            const double dR1 = (FRh[j * NVAR + k] - FRh[(j - 1) * NVAR + k]);
            const double dR2 = (FRh[(j + 1) * NVAR + k] - FRh[j * NVAR + k]);"""),
    "full step over half the dt":
        ("(H[j * NVAR + k] - H[(j - 1) * NVAR + k]) / dh * dt;",
         "(H[j * NVAR + k] - H[(j - 1) * NVAR + k]) / dh * (dt / 2.0);"),
    "boundary flux taken from the first-order flux":
        ("hface[i * NVAR + k] = H[(i + GHOST - 1) * NVAR + k];",
         "hface[i * NVAR + k] = G[(i + GHOST - 1) * NVAR + k];"),
}

PINS = [
    "test_vanleer_closed_form",
    "test_split_fluxes_closed_form",
    "test_cfl_uniform_closed_form",
    "test_uniform_state_bitwise",
    "test_one_d_embedded_and_axis_permutation",
    "test_mirror_symmetry_bitwise",
    "test_transpose_reverses_sweep_order",
    "test_decomposition_invariance_bitwise",
    "test_conservation_periodic",
    "test_flux_uniform_closed_form",
    "test_flux_one_d_closed_form",
    "test_flux_patch_conservation",
    "test_flux_shared_faces_bitwise",
    "test_pressureless_advection",
    "test_acoustic_wave_second_order",
    "test_sod_against_exact_riemann",
    "test_pencil_against_mpmath_reference",
]

RUNNER = r"""
import sys, inspect
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import oracle
oracle.use_library({lib!r})
import test_oracle_pins as P
failed = []
for name in {pins!r}:
    fn = getattr(P, name)
    params = inspect.signature(fn).parameters
    try:
        if params:
            fn(**{{k: v for k, v in dict(n=8, order=1).items() if k in params}})
        else:
            fn()
    except Exception as e:  # an assertion, a NaN comparison, anything
        failed.append(name)
        break
print("FAILED_PINS", failed)
"""


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    old, new = MUTANTS[name]
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, "mutation anchor must occur exactly once"
    with tempfile.TemporaryDirectory() as tmp:
        msrc = os.path.join(tmp, "mutant.c")
        with open(msrc, "w") as f:
            f.write(src.replace(old, new))
        lib = oracle.build(src=msrc, out=os.path.join(tmp, "libmutant.so"))
        code = RUNNER.format(root=ROOT, tests=HERE, lib=lib, pins=PINS)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                           timeout=600)
    caught = r.returncode != 0 or ("FAILED_PINS []" not in r.stdout)
    assert caught, "no pin caught the planted mistake: " + name


@pytest.mark.slow
def test_unmodified_oracle_passes_every_pin():
    """Control for the cases above: the real oracle passes the same runner."""
    code = RUNNER.format(root=ROOT, tests=HERE, lib=oracle._load()._name, pins=PINS)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0 and "FAILED_PINS []" in r.stdout, r.stdout + r.stderr
