"""Mistakes planted in copies of the oracle's C source must fail a pin.

Each case below replaces one expression of oracle/rmp_oracle.c by a plausible
wrong one (a factor of the solvent mass m or of kT dropped, a square root
misplaced, a term left out), compiles the copy with the oracle's own flags into
a separate library, and runs the named pin against it: the pin has to fail.
The original source has to pass the same pins (test_oracle_pins.py runs them).
All of this runs on the CPU.
"""
import pytest

import oracle
import test_oracle_pins as pins

# (name, original text, planted text, pin, pin arguments)
MUTANTS = [
    ("solvent kick dt/2 instead of dt/(2m)",
     "s->h = (0.5 * p->dt) / p->mass;", "s->h = (0.5 * p->dt);",
     pins.test_momentum_and_energy_with_colloids_at_nonunit_mass, ()),
    ("colloid kick dt/2 instead of dt/(2M)",
     "s->hc[c] = (0.5 * p->dt) / p->cmass[c];", "s->hc[c] = (0.5 * p->dt);",
     pins.test_momentum_and_energy_with_colloids_at_nonunit_mass, ()),
    ("initial velocities scaled by sqrt(kT) instead of sqrt(kT/m)",
     "double sc = sqrt(p->kT / p->mass);", "double sc = sqrt(p->kT);",
     pins.test_init_maxwellian_at_nonunit_mass_and_temperature, ()),
    ("kinetic energy without the mass",
     "o->ke_solvent = 0.5 * s->p.mass * ke;", "o->ke_solvent = 0.5 * ke;",
     pins.test_init_maxwellian_at_nonunit_mass_and_temperature, ()),
    ("temperature equation without the factor m",
     "tterm[c] = (s->p.mass * tsum) / (double)(nn - 1);", "tterm[c] = tsum / (double)(nn - 1);",
     pins.test_temperature_equation_returns_kT, ("srd",)),
    ("thermostat noise N(0, kT) instead of N(0, kT/m)",
     "const double sc = sqrt(s->p.kT / s->p.mass);", "const double sc = sqrt(s->p.kT);",
     pins.test_anderson_thermostat_draws_relative_velocities_at_kT, ()),
    ("thermostat without the cell mean of the draws removed",
     "s->v[d][j] = u[d] + ((sc * z[d]) - gm[d]);", "s->v[d][j] = u[d] + (sc * z[d]);",
     pins.test_anderson_thermostat_draws_relative_velocities_at_kT, ()),
    ("virtual momentum without sqrt(kT/m)",
     "const double sc = sqrt(s->p.kT / s->p.mass);", "const double sc = 1.0;",
     pins.test_virtual_particles_carry_thermal_momentum_at_kT, ()),
    ("virtual momentum variance (n0-n)^2 instead of (n0-n)",
     "const double sd = sqrt((double)(n0 - nn)) * sc;", "const double sd = (double)(n0 - nn) * sc;",
     pins.test_virtual_particles_carry_thermal_momentum_at_kT, ()),
    ("virtual fill averaged over n instead of n0",
     "u[d] = (S[d] + (sd * z[d])) / (double)n0;", "u[d] = (S[d] + (sd * z[d])) / (double)nn;",
     pins.test_virtual_particles_carry_thermal_momentum_at_kT, ()),
]


@pytest.mark.parametrize("name,orig,planted,pin,args", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, name, orig, planted, pin, args):
    src = oracle.source()
    assert src.count(orig) == 1, f"expression to mutate not found once: {orig}"
    so = oracle.compile_variant(src.replace(orig, planted), str(tmp_path / "liboracle_mut.so"))
    with oracle.using(so):
        with pytest.raises(AssertionError):
            pin(*args)


def test_unplanted_copy_passes_the_same_pins(tmp_path):
    """The copy path itself is sound: the unaltered source, compiled the same
    way, passes every pin used above."""
    so = oracle.compile_variant(oracle.source(), str(tmp_path / "liboracle_copy.so"))
    with oracle.using(so):
        done = set()
        for _, _, _, pin, args in MUTANTS:
            if (pin, args) in done:
                continue
            done.add((pin, args))
            pin(*args)
