"""Planted mistakes in the oracle, on the CPU: each replaces one oracle
function by a plausible wrong version (a dropped factor, a wrong sign or
exponent, swapped axes or bits, a reversed rule) and checks that at least one
of the pins written against the paper and the mathematics then fails. A
mistake no pin catches fails this test."""
import math

import numpy as np
import pytest

import test_oracle_csg as pins_csg
import test_oracle_multires as pins_mr
import test_oracle_pins as pins
import test_oracle_register as pins_reg
from oracle import cells, csg, force, geometry, hvp, kernel, metrics, multires, neighbors, register, step


def _fails(pin_calls):
    """True if any of the pins raises AssertionError (or a numerical error)."""
    for fn, args in pin_calls:
        try:
            fn(*args)
        except (AssertionError, FloatingPointError, ValueError, IndexError):
            return True
    return False


def _wrap(orig, post):
    return lambda *a, **k: post(orig(*a, **k))


MUTATIONS = {
    # Eq. 17: the printed 3-D constant instead of the normalising one
    "alpha_printed": (kernel, "alpha", lambda h, d=3: 21.0 / (6.0 * math.pi * h ** 3) if d == 3 else 7.0 / (4.0 * math.pi * h * h),
                      [(pins.test_kernel_3d_normalised_and_printed_constant_is_not, ())]),
    # Eq. 16 with the third power of (1 - q/2)
    "W_cubed": (kernel, "W", lambda r, h, d=3: kernel.alpha(h, d) * np.clip(1 - 0.5 * np.asarray(r) / h, 0, None) ** 3
                * (2 * np.asarray(r) / h + 1),
                [(pins.test_kernel_3d_normalised_and_printed_constant_is_not, ()),
                 (pins.test_dW_dr_matches_central_difference, ())]),
    # the pair-force coefficient with h instead of h^2
    "force_coef_h": (force, "force_coef", lambda h: 5.0 * kernel.alpha(h, 3) / h,
                     [(pins.test_two_particle_force_is_minus_kernel_gradient, ())]),
    # the neighbour distance without its z term
    "pair_d2_no_z": (neighbors, "pair_d2", lambda a, b: np.float32(
        np.float32((a[..., 0] - b[..., 0]) ** 2) + np.float32((a[..., 1] - b[..., 1]) ** 2)),
                     [(pins.test_neighbors_equal_kdtree_search, ())]),
    # the rank rule reversed: sources of higher rank act
    "rank_reversed": (force, "RANK", np.array([3, 2, 1, 0, 0], np.int64),
                      [(pins.test_class_interaction_rule, ())]),
    # dt^2 with h/8
    "time_step_h8": (step, "time_step", _wrap(step.time_step, lambda t: 2.0 * t),
                     [(pins.test_step_moves_fastest_particle_exactly_h_over_16, ())]),
    # inside and outside swapped
    "winding_flipped": (geometry, "winding_number", _wrap(geometry.winding_number, lambda w: 1.0 - w),
                        [(pins.test_signed_distance_matches_analytic_box, ())]),
    # the pair Jacobian with the wrong sign of its r r^T term
    "jacobian_sign": (hvp, "pair_jacobian", lambda r, h: _jac_plus(r, h),
                      [(pins.test_jvp_matches_central_difference_of_force, ())]),
    # the residual of the unprojected acceleration
    "residual_unprojected": (metrics, "projected_accel", lambda wl, a, owner, feat_seg, tag=None: np.array(a, float),
                             [(pins.test_residual_closed_form_on_cube_face_edge_and_volume, ())]),
    # cell keys with x and y exchanged
    "key_xy_swapped": (cells, "linear_key", lambda c, dims, slab: cells.__dict__["_orig_linear_key"](
        c[:, [1, 0, 2]], [dims[1], dims[0], dims[2]], slab),
                       [(pins.test_cell_keys_contain_particles_and_order_is_key_then_id, ())]),
    # Eq. 9 with the y and z bits exchanged
    "morton_yz": (register, "morton", lambda x, y, z, bits=21: register.__dict__["_orig_morton"](x, z, y, bits),
                  [(pins_reg.test_morton_codes_by_hand, ())]),
    # the centre child of a four-way split forgotten
    "subdivision_no_centre": (register, "children", lambda a, b, c, cell: (
        lambda ch: ch[:3] if ch is not None and len(ch) == 4 else ch)(register.__dict__["_orig_children"](a, b, c, cell)),
                              [(pins_reg.test_child_counts_of_the_three_split_patterns, ()),
                               (pins_reg.test_subdivision_tiles_every_facet, (1,))]),
    # the particles' levels ignored (every pair at the coarse length)
    "mr_levels_ignored": (multires, "accel", lambda wl, level, *a, **k: multires.__dict__["_orig_accel"](
        wl, np.minimum(np.asarray(level), 0) if np.any(np.asarray(level) > 0) else level, *a, **k),
                 [(pins_mr.test_two_particles_of_different_levels, ()),
                  (pins_mr.test_halving_every_length_scales_the_force_by_sixteen, ())]),
    # a union foot accepted inside another part
    "csg_union_inside": (csg, "on_boundary", lambda p, facets, geo, margin=1e-9: (
        np.ones(len(np.atleast_2d(p)), bool), np.zeros(len(np.atleast_2d(p)), bool)),
                         [(pins_csg.test_projection_lands_on_the_combined_box, ("union",))]),
}


def _jac_plus(r, h):
    d = np.linalg.norm(r, axis=1)
    t = np.clip(1.0 - d / (2.0 * h), 0.0, None)
    K = kernel.force_coef(1.0) / h ** 5
    safe = np.where(d > 0, d, 1.0)
    rr = np.einsum("pi,pj->pij", r, r) / safe[:, None, None]
    eye = np.eye(3)[None]
    return K[:, None, None] * (t[:, None, None] ** 3 * eye
                               + (3.0 / (2.0 * h))[:, None, None] * t[:, None, None] ** 2 * rr)


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    mod, attr, repl, pin_calls = MUTATIONS[name]
    # the replacements that call the original reach it under a private name
    monkeypatch.setitem(cells.__dict__, "_orig_linear_key", cells.linear_key)
    monkeypatch.setitem(register.__dict__, "_orig_morton", register.morton)
    monkeypatch.setitem(multires.__dict__, "_orig_accel", multires.accel)
    monkeypatch.setitem(register.__dict__, "_orig_children", register.children)
    # every module that imported the function by name sees the mistake too
    orig = mod.__dict__[attr]
    for m in (kernel, force, step, hvp, metrics, geometry, neighbors, cells, register, multires, csg,
              pins, pins_reg, pins_mr, pins_csg):
        if m is mod or (attr in m.__dict__ and m.__dict__[attr] is orig):
            monkeypatch.setattr(m, attr, repl)
    assert _fails(pin_calls), f"no pin caught the planted mistake {name}"
