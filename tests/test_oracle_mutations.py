"""Each pin can fail: a plausible mistake planted in the LBM oracle's core
steps (collision, equilibrium, moving walls, fiber bounce-back, momentum
exchange, free-slip reflection, refill, stabilization, side walls, cell
mapping, rigid step, contacts, periodic images, external loads) makes
the named pins fail (the rest of the suite runs every pin with none
planted).  The planted mistakes of the coupled rigid-body update are in
test_oracle_coupling_pins.py."""
import pytest

from oracle import pyoracle as O

import test_oracle_freeslip as FS
import test_oracle_pins as P

MUTATIONS = {
    5: ("odd part relaxed with omega_e",
        [P.test_trt_rates_act_on_even_and_odd_parts, P.test_collision_conserves_mass_and_momentum,
         lambda: P.test_stabilized_total_momentum_decays_by_one_minus_omega_odd(0.8, False)]),
    6: ("3 instead of 9/2 for (c.u)^2 in f_eq",
        [P.test_equilibrium_moments, P.test_equilibrium_even_odd_split]),
    7: ("collision's even equilibrium without (c.u)^2",
        [P.test_collision_conserves_mass_and_momentum, lambda: P.test_mass_conservation(False, 0.01),
         P.test_closed_box_conserves_mass_and_stops]),
    8: ("moving-wall term with the wrong sign", [P.test_couette_closed_form]),
    9: ("fiber bounce-back without the surface velocity",
        [P.test_external_force_enters_the_momentum_budget,
         P.test_stabilized_momentum_budget_with_a_forced_particle]),
    10: ("link force without its factor 2",
         [P.test_external_force_enters_the_momentum_budget, P.test_drag_balance_fixed_fiber]),
    11: ("torque as dF x r", [P.test_force_and_torque_signs]),
    12: ("free-slip walls bouncing back",
         [lambda: FS.test_free_slip_box_is_half_of_the_mirrored_periodic_box("x", False),
          FS.test_body_force_along_free_slip_walls_accelerates_uniformly]),
    13: ("refill at the new pose and motion", [P.test_refill_uses_each_old_owners_rigid_motion_at_its_old_pose]),
    14: ("stabilization shift added instead of subtracted",
         [lambda: P.test_stabilized_total_momentum_decays_by_one_minus_omega_odd(0.8, False),
          P.test_stabilized_momentum_with_body_force_reaches_its_fixed_point]),
    15: ("resting side wall returns the population in its own direction",
         [P.test_closed_box_conserves_mass_and_stops]),
    16: ("cylinder's axial bound at L instead of L/2",
         [P.test_mapping_hand_counted, P.test_mapping_volume_converges]),
    17: ("axis of the conjugate quaternion",
         [P.test_mapping_hand_counted, P.test_quaternion_update_constant_rotation,
          P.test_free_precession_conserves_angular_momentum]),
    18: ("highest id keeps a cell claimed twice", [P.test_mapping_overlap_lowest_id_wins]),
    19: ("spherocylinder caps centred at the cylinder's ends",
         [P.test_spherocylinder_predicate_is_the_distance_to_the_axis_segment,
          P.test_spherocylinder_cell_count_converges_to_its_volume]),
    20: ("explicit rigid step moving with the old velocity", [P.test_rigid_translation_and_wrap]),
    21: ("I_par and I_perp swapped in the inverse inertia",
         [P.test_free_precession_conserves_angular_momentum, P.test_quaternion_update_constant_rotation]),
    22: ("attractive contact force",
         [P.test_contact_side_by_side_closed_form, P.test_contact_is_a_central_pair_force]),
    23: ("contact torque on q about the centre of p", [P.test_contact_is_a_central_pair_force]),
    24: ("no minimum image across periodic faces", [P.test_mapping_periodic_translation]),
    25: ("mean velocity over all cells, solid ones included",
         [P.test_mean_velocity_is_the_fluid_cell_mean, P.test_stabilized_momentum_budget_with_a_forced_particle]),
    26: ("spherocylinder caps' inertia without the parallel-axis shift",
         [lambda: P.test_body_mass_and_inertia_by_quadrature("spherocylinder")]),
    27: ("external force dropped",
         [P.test_external_force_enters_the_momentum_budget,
          lambda: P.test_external_load_enters_the_first_explicit_step("cylinder")]),
    28: ("external torque dropped", [lambda: P.test_external_load_enters_the_first_explicit_step("spherocylinder")]),
}


@pytest.mark.parametrize("code", sorted(MUTATIONS))
def test_pins_fail_on_planted_mistakes(code):
    what, pins = MUTATIONS[code]
    try:
        O.set_mutation(code)
        for pin in pins:
            with pytest.raises(AssertionError):
                pin()
    finally:
        O.set_mutation(0)
