"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source, builds the
copy with the oracle's own flags, and runs the pins that cover that part of
the oracle against it in a child process (PIC_ORACLE_LIB points the wrapper
at the copy).  The pins must fail on every mutant; on the unmodified source
they pass (they are part of the ordinary suite).  The mistakes:

* absorbed energy taken at v^{n-1/2} instead of v^{n+1/2}, or without v_x, v_y
  ("Boundary energy diagnostics", eqs. 3-8);
* a newborn beyond the anode dropped without its tally;
* initial positions on half the gap, or ions loaded at the electron
  temperature ("Model": uniform load, Maxwellian at T_e0, T_i0);
* replenished electron and ion at independent positions, on half the gap,
  or the ion at the electron temperature ("Model": pairs at overlapping
  random positions with Maxwellian velocities).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

from oracle import build_oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TALLIES = "tests/test_oracle_tallies.py"

MUTANTS = [
    ("energy at the previous half step",
     "tally_abs(o, sp, m->fate - 1, m->v[0], m->v[1], m->v[2]);",
     "tally_abs(o, sp, m->fate - 1, m->v[0], m->v[1], s->vz[p]);",
     TALLIES + "::test_absorbed_energy_is_full_3v_energy_at_crossing"),
    ("energy without v_x, v_y",
     "tally_abs(o, sp, m->fate - 1, m->v[0], m->v[1], m->v[2]);",
     "tally_abs(o, sp, m->fate - 1, 0.0, 0.0, m->v[2]);",
     TALLIES + "::test_absorbed_energy_is_full_3v_energy_at_crossing"),
    ("newborn beyond the anode not tallied",
     "if (z >= c->L) { tally_abs(o, sp, 1, vx, vy, vz); return 0; }",
     "if (z >= c->L) { return 0; }",
     TALLIES + "::test_newborn_beyond_the_anode_is_absorbed_at_once"),
    ("load on half the gap",
     "S->z[p] = c->L * o_u53(b1[0], b1[1]);",
     "S->z[p] = 0.5 * c->L * o_u53(b1[0], b1[1]);",
     TALLIES + "::test_initial_load_uniform_and_maxwellian"),
    ("ions loaded at the electron temperature",
     "        double T = (s == OSP_I) ? c->Ti0 : c->Te0;\n        double sig",
     "        double T = c->Te0;\n        double sig",
     TALLIES + "::test_initial_load_uniform_and_maxwellian"),
    ("pair at independent positions",
     "if (birth(o, OSP_I, idi, z, si * a1, si * a2, si * a3)) return -1;",
     "if (birth(o, OSP_I, idi, c->L * o_u53(i0[0], i0[3]), si * a1, si * a2, si * a3)) return -1;",
     TALLIES + "::test_replenished_pairs_share_position_and_are_maxwellian"),
    ("pairs on half the gap",
     "double z = c->L * o_u53(e1[0], e1[1]);",
     "double z = 0.5 * c->L * o_u53(e1[0], e1[1]);",
     TALLIES + "::test_replenished_pairs_share_position_and_are_maxwellian"),
    ("replenished ion at the electron temperature",
     "si = sqrt(Q_E * c->Ti0 / d->mass[OSP_I]);",
     "si = sqrt(Q_E * c->Te0 / d->mass[OSP_I]);",
     TALLIES + "::test_replenished_pairs_share_position_and_are_maxwellian"),
]


def _build_mutant(tmp, k, old, new):
    src = open(build_oracle.SRC).read()
    assert src.count(old) == 1, "mutation site not unique: %r" % old
    d = os.path.join(tmp, "m%d" % k)
    os.makedirs(d)
    with open(os.path.join(d, "pic_oracle.c"), "w") as f:
        f.write(src.replace(old, new))
    hdr = os.path.join(os.path.dirname(build_oracle.SRC), "pic_oracle.h")
    with open(os.path.join(d, "pic_oracle.h"), "w") as f:
        f.write(open(hdr).read())
    lib = os.path.join(d, "liboracle.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-D_GNU_SOURCE",
                           "-o", lib, os.path.join(d, "pic_oracle.c"), "-lm"])
    return lib


def _run_pins(lib, nodeid):
    env = dict(os.environ, PIC_ORACLE_LIB=lib)
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", nodeid],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)


def test_pins_fail_on_planted_mistakes(tmp_path):
    libs = [_build_mutant(str(tmp_path), k, old, new) for k, (_, old, new, _) in enumerate(MUTANTS)]
    with ThreadPoolExecutor(max_workers=4) as ex:
        runs = list(ex.map(lambda a: _run_pins(*a), [(lib, m[3]) for lib, m in zip(libs, MUTANTS)]))
    survived = []
    for (name, _, _, nodeid), r in zip(MUTANTS, runs):
        # exit status 1: the pins ran and failed (2 and above: collection or usage errors)
        if r.returncode != 1:
            survived.append("%s: pytest exit %d\n%s" % (name, r.returncode, r.stdout[-600:]))
    assert not survived, "\n".join(survived)


def test_pins_pass_on_the_unmodified_source(tmp_path):
    # the same copy-and-build route with no change: guards the harness itself
    lib = _build_mutant(str(tmp_path), 99, "#include <math.h>", "#include <math.h>")
    r = _run_pins(lib, TALLIES)
    assert r.returncode == 0, r.stdout[-1500:]
