"""The pins must reject a wrong oracle.

Each case plants one plausible mistake (a dropped term, a wrong sign, index
or constant, a transposed operand, the Mul22 typo as printed) in a copy of
``oracle.c``, builds the copy with the same flags, and checks that at least
one of the pins aimed at that part of the oracle fails on it.  Everything
runs on the CPU; the real oracle is never modified.
"""
import os

import pytest

import oracle
import test_oracle_operators as OPS
import test_oracle_accurate_add as ACC
import test_oracle_accurate_mul_div as AMD
import test_oracle_compensated as CMP
import test_oracle_convert as CNV
import test_oracle_dot_backward as DBW
import test_oracle_golden as GOLD
import test_oracle_horner as HOR
import test_oracle_paper_tables as TAB
import test_oracle_primitives as PRIM
import test_oracle_reductions as RED

_SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

PRIM_PINS = [
    lambda: PRIM.test_add12_is_exact_and_rounds_like_ieee(-40, 40),
    PRIM.test_add12_sterbenz_pairs_have_zero_error,
    PRIM.test_split_exhaustive_unit_binade,
    lambda: PRIM.test_mul12_is_exact(False, -50, 50),
    lambda: PRIM.test_mul12_is_exact(True, -50, 50),
]
OP_PINS = [
    OPS.test_add22_zero_low_words_is_the_exact_add12_pair,
    OPS.test_add22_identities,
    lambda: OPS.test_add22_error_bound("mixed", "add"),
    lambda: OPS.test_add22_error_bound("near", "add"),
    lambda: OPS.test_mul22_zero_low_words_is_the_exact_product_pair(False),
    lambda: OPS.test_mul22_relative_error_bound("random", False),
    OPS.test_div22_identities,
    lambda: OPS.test_div22_relative_error_bound("random", False),
]
RED_PINS = [
    lambda: RED.test_exact_dot_rounds_to_fsum(-20, 20),
    RED.test_exact_dot_brute_force_and_extremes,
    RED.test_dot_seq_single_term_is_the_exact_product_pair,
    lambda: RED.test_dot_seq_error_bound(1000),
    RED.test_gemm_identity_returns_a,
    RED.test_gemm_block_and_exact_entries,
]
TAB_PINS = [
    lambda: TAB.test_f32_add_mul_match_numpy("add"),
    lambda: TAB.test_f32_add_mul_match_numpy("mul"),
    TAB.test_f32_mad_is_a_single_rounding,
    lambda: TAB.test_ff_errors_against_fractions("add22"),
    lambda: TAB.test_ff_errors_against_fractions("mul22"),
    TAB.test_ff_errors_edge_cases,
]
ACC_PINS = [
    ACC.test_zero_low_words_is_the_exact_add12_pair,
    ACC.test_identities,
    lambda: ACC.test_relative_error_bound_holds_under_cancellation("cancel"),
    lambda: ACC.test_relative_error_bound_holds_under_cancellation("random"),
    lambda: ACC.test_relative_error_bound_holds_under_cancellation("gap"),
]
AMD_PINS = [
    AMD.test_mul_zero_low_words_is_the_exact_product_pair,
    AMD.test_mul_identities,
    AMD.test_div_identities,
    AMD.test_hand_derived_cases,
    lambda: AMD.test_mul_relative_error_bound("random"),
    lambda: AMD.test_div_relative_error_bound("random"),
    lambda: AMD.test_div_relative_error_bound("near"),
    lambda: AMD.test_ff_errors_against_fractions("div22"),
]
HOR_PINS = [
    HOR.test_degree_zero_returns_the_constant,
    HOR.test_integer_polynomials_are_exact,
    lambda: HOR.test_binomial_closed_form(7),
    lambda: HOR.test_random_polynomials(8),
    HOR.test_compensated_is_as_if_twice_the_precision,
    HOR.test_float_float_coefficients_and_points,
]
CNV_PINS = [
    CNV.test_from_f64_rounds_hi_and_keeps_48_bits,
    CNV.test_from_f64_of_binary32_values_is_exact,
    CNV.test_to_f64_rounds_once,
    CNV.test_round_trip_where_the_bits_fit,
]
DBW_PINS = [
    DBW.test_power_of_two_gradients_are_exact_and_segment_correctly,
    DBW.test_general_gradients_within_the_mul22_bound,
]
CMP_PINS = [
    CMP.test_empty_and_single_terms,
    CMP.test_integer_data_is_exact,
    lambda: CMP.test_dot2_error_bound_ill_conditioned(25),
    lambda: CMP.test_dot2_error_bound_ill_conditioned(40),
    CMP.test_dot2_where_the_naive_sum_fails,
    lambda: CMP.test_sum2_error_bound_random(3000),
]

# Evaluation-order pins: the hand-derived cases whose results change when a
# chain is regrouped (the regression lock, written by the oracle itself, is
# deliberately not among them).
ORDER_PINS = {op: [lambda op=op: GOLD.check_hand_cases(op)]
              for op in ("add22", "mul22", "div22", "horner_comp")}

# (name, original text, planted text, pins expected to catch it)
MUTATIONS = [
    ("add22_order_first_arm", "s = (((ah - r) + bh) + bl) + al;",
     "s = (((ah - r) + bh) + al) + bl;", ORDER_PINS["add22"]),
    ("add22_order_second_arm", "s = (((bh - r) + ah) + al) + bl;",
     "s = (((bh - r) + ah) + bl) + al;", ORDER_PINS["add22"]),
    ("mul22_order_t2_first", "float t3 = ((ah * bl) + (al * bh)) + t2;",
     "float t3 = (t2 + (ah * bl)) + (al * bh);", ORDER_PINS["mul22"]),
    ("mul22_order_t2_with_al_bh", "float t3 = ((ah * bl) + (al * bh)) + t2;",
     "float t3 = (t2 + (al * bh)) + (ah * bl);", ORDER_PINS["mul22"]),
    ("div22_order_al_before_uu", "float t = (((ah - u) - uu) + al) - (c * bl);",
     "float t = (((ah - u) + al) - uu) - (c * bl);", ORDER_PINS["div22"]),
    ("div22_order_u_plus_uu", "float t = (((ah - u) - uu) + al) - (c * bl);",
     "float t = ((ah - (u + uu)) + al) - (c * bl);", ORDER_PINS["div22"]),
    ("horner_comp_order_pi_first", "            r = (r * xk) + (pi + sigma);",
     "            r = ((r * xk) + pi) + sigma;", ORDER_PINS["horner_comp"]),
    ("horner_comp_order_sigma_first", "            r = (r * xk) + (pi + sigma);",
     "            r = ((r * xk) + sigma) + pi;", ORDER_PINS["horner_comp"]),
    ("add12_error_sign", "float r = (a - (s - v)) + (b - v);",
     "float r = (a - (s - v)) - (b - v);", PRIM_PINS),
    ("add12_wrong_operand", "float v = s - a;", "float v = s - b;", PRIM_PINS),
    ("split_constant", "const float c_split = 4097.0f;", "const float c_split = 4096.0f;",
     PRIM_PINS),
    ("split_low_word", "    *lo_out = a - hi;", "    *lo_out = a - scaled;", PRIM_PINS),
    ("split_uncancelled", "const float hi = scaled - (scaled - a);",
     "const float hi = scaled - a;", PRIM_PINS),
    ("dekker_transposed_term", "rem = rem - (a2 * b1);",
     "rem = rem - (a1 * b2);", PRIM_PINS),
    ("fma_sign", "*y_out = fmaf(a, b, -x);", "*y_out = fmaf(a, b, x);", PRIM_PINS),
    ("add22_branch_flipped", "if (fabsf(ah) >= fabsf(bh))", "if (fabsf(ah) <= fabsf(bh))",
     OP_PINS),
    ("add22_dropped_low_word", "s = (((ah - r) + bh) + bl) + al;",
     "s = (((ah - r) + bh) + bl);", OP_PINS),
    ("mul22_printed_typo", "add12(t1, t3, rh, rl);", "add12(t1, t2, rh, rl);", OP_PINS),
    ("mul22_wrong_index", "float t3 = ((ah * bl) + (al * bh)) + t2;",
     "float t3 = ((ah * bl) + (al * bl)) + t2;", OP_PINS),
    ("div22_sign", "float t = (((ah - u) - uu) + al) - (c * bl);",
     "float t = (((ah - u) - uu) + al) + (c * bl);", OP_PINS),
    ("div22_dropped_term", "float t = (((ah - u) - uu) + al) - (c * bl);",
     "float t = ((ah - u) + al) - (c * bl);", OP_PINS),
    ("exact_shift", "mag <<= (pos % 32);", "mag <<= (pos % 31);", RED_PINS),
    ("exact_exponent", "*e = ex - 24;", "*e = ex - 23;", RED_PINS),
    ("dot_dropped_error_term", "        add22(acc_h, acc_l, p, e, &acc_h, &acc_l);",
     "        add22(acc_h, acc_l, p, 0.0f, &acc_h, &acc_l);", RED_PINS),
    ("accurate_dropped_tl", "    float w = tl + vl;", "    float w = vl;", ACC_PINS),
    ("accurate_sign", "    float c = sl + th;", "    float c = sl - th;", ACC_PINS),
    ("accurate_low_pair", "    add12(al, bl, &th, &tl);", "    add12(al, bh, &th, &tl);", ACC_PINS),
    ("accurate_final_order", "    fast_add12(vh, w, rh, rl);", "    fast_add12(w, vh, rh, rl);", ACC_PINS),
    ("mulacc_dropped_tl0", "    float tl1 = fmaf(ah, bl, tl0);", "    float tl1 = fmaf(ah, bl, 0.0f);",
     AMD_PINS),
    ("mulacc_wrong_index", "    float cl2 = fmaf(al, bh, tl1);", "    float cl2 = fmaf(al, bl, tl1);",
     AMD_PINS),
    ("mulacc_dropped_cl1", "    float cl3 = cl1 + cl2;", "    float cl3 = cl2;", AMD_PINS),
    ("divacc_residual_sign", "    float el0 = -bl * th;", "    float el0 = bl * th;", AMD_PINS),
    ("divacc_newton_sign", "    float eh0 = fmaf(-bh, th, 1.0f);", "    float eh0 = fmaf(bh, th, -1.0f);",
     AMD_PINS),
    ("divacc_dropped_low", "    float v = dl2 + sl;", "    float v = sl;", AMD_PINS),
    ("divacc_dropped_ml", "    mul22_accurate(ah, al, mh, ml, rh, rl);",
     "    mul22_accurate(ah, al, mh, 0.0f, rh, rl);", AMD_PINS),
    ("divacc_dropped_el", "    float dl = fmaf(el, th, dl1);", "    float dl = dl1;", AMD_PINS),
    ("errors_div_cross_term", "            la_add_product(&err, rl[i], bh[i]);\n",
     "", AMD_PINS),
    ("horner_order", "            s = (s * x[k]) + a[i];", "            s = (s + a[i]) * x[k];", HOR_PINS),
    ("horner_comp_dropped_pi", "            r = (r * xk) + (pi + sigma);",
     "            r = (r * xk) + sigma;", HOR_PINS),
    ("horner_comp_dropped_sigma", "            r = (r * xk) + (pi + sigma);",
     "            r = (r * xk) + pi;", HOR_PINS),
    ("horner_comp_unscaled_r", "            r = (r * xk) + (pi + sigma);",
     "            r = r + (pi + sigma);", HOR_PINS),
    ("horner_comp_no_correction", "        y[k] = s + r;", "        y[k] = s;", HOR_PINS),
    ("horner_ff_coefficient_lo", "            add22(ph, pl, ah[i], al[i], &sh, &sl);",
     "            add22(ph, pl, ah[i], 0.0f, &sh, &sl);", HOR_PINS),
    ("horner_ff_point_lo", "            mul22(sh, sl, xh[k], xl[k], 0, &ph, &pl);",
     "            mul22(sh, sl, xh[k], 0.0f, 0, &ph, &pl);", HOR_PINS),
    ("horner_ff_top_lo", "        float sh = ah[degree], sl = al[degree];",
     "        float sh = ah[degree], sl = 0.0f;", HOR_PINS),
    ("from_f64_low_word_in_binary32", "        lo[i] = (float)(x[i] - (double)h);",
     "        lo[i] = (float)x[i] - h;", CNV_PINS),
    ("to_f64_binary32_sum", "        x[i] = (double)hi[i] + (double)lo[i];",
     "        x[i] = (double)(hi[i] + lo[i]);", CNV_PINS),
    ("dot_bwd_swapped_operands", "            mul22(gh[v], gl[v], yh[i], yl[i], 0, &dxh[i], &dxl[i]);",
     "            mul22(gh[v], gl[v], xh[i], xl[i], 0, &dxh[i], &dxl[i]);", DBW_PINS),
    ("dot_bwd_neighbour_gradient", "            mul22(gh[v], gl[v], xh[i], xl[i], 0, &dyh[i], &dyl[i]);",
     "            mul22(gh[v > 0 ? v - 1 : v], gl[v], xh[i], xl[i], 0, &dyh[i], &dyl[i]);", DBW_PINS),
    ("dot_bwd_dropped_low_word", "            mul22(gh[v], gl[v], yh[i], yl[i], 0, &dxh[i], &dxl[i]);",
     "            mul22(gh[v], gl[v], yh[i], 0.0f, 0, &dxh[i], &dxl[i]);", DBW_PINS),
    ("dot_bwd_no_zero_fill", "        dxh[i] = dxl[i] = dyh[i] = dyl[i] = 0.0f;",
     "        dxh[i] = dxl[i] = dyh[i] = dyl[i] = 1.0f;", DBW_PINS),
    ("dot2_dropped_product_error", "        s = s + (q + r);", "        s = s + q;", CMP_PINS),
    ("dot2_dropped_sum_error", "        s = s + (q + r);", "        s = s + r;", CMP_PINS),
    ("sum2_dropped_error", "        s = s + q;\n    }\n    out2[0] = p;\n    out2[1] = s;\n}\n\nvoid oracle_dot2",
     "        s = s + 0.0f * q;\n    }\n    out2[0] = p;\n    out2[1] = s;\n}\n\nvoid oracle_dot2", CMP_PINS),
    ("dot2_first_term_error", "        mul12_fma(x[0], y[0], &p, &s);", "        { mul12_fma(x[0], y[0], &p, &s); s = 0.0f; }", CMP_PINS),
    ("mad_unfused", "r[i] = fmaf(a[i], b[i], c[i]);", "r[i] = a[i] * b[i] + c[i];",
     TAB_PINS),
    ("errors_dropped_low_word", "            la_add_f32(&exact, bl[i], 1);\n            la_add_f32(&lo, al[i], 1);",
     "            la_add_f32(&lo, al[i], 1);", TAB_PINS),
    ("errors_mul22_cross_term", "            la_add_product(&exact, al[i], bh[i]);\n            la_add_product(&exact, al[i], bl[i]);",
     "            la_add_product(&exact, al[i], bh[i]);\n            la_add_product(&exact, al[i], bh[i]);", TAB_PINS),
    ("errors_bound_exponent", "double b1 = ldexp(lo_mag, -24), b2 = ldexp(big, -44);",
     "double b1 = ldexp(lo_mag, -24), b2 = ldexp(big, -45);", TAB_PINS),
    ("gemm_transposed_stride", "Bh + j, Bl + j,\n                              ldb, K, out);",
     "Bh + j, Bl + j,\n                              1, K, out);", RED_PINS),
]


@pytest.mark.parametrize("name,orig,planted,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_reject_planted_mistake(tmp_path, name, orig, planted, pins):
    src = open(_SRC).read()
    assert src.count(orig) == 1, f"mutation anchor for {name} not unique"
    mutated = tmp_path / "oracle_mut.c"
    mutated.write_text(src.replace(orig, planted))
    so = oracle.build(force=True, src=str(mutated), out=str(tmp_path / "liboracle_mut.so"))
    caught = []
    with oracle.using_library(so):
        for pin in pins:
            try:
                pin()
            except (AssertionError, ValueError, ZeroDivisionError, OverflowError):
                caught.append(pin)
                break
    assert caught, f"no pin rejects the planted mistake {name}"
