"""Mutation check of the oracle's pins.

Each case plants one plausible mistake (a dropped term, a wrong sign, a wrong
or transposed index, a missing conjugate, a wrong rounding rule) in a copy of
`oracle/su3_oracle.c`, compiles the copy into a temporary library on the CPU,
and runs the oracle pins against it. Every mutant must fail at least one pin;
a mutant that passes them all would mean the pins cannot tell that mistake
from the paper's definition.
"""

import importlib.util
import inspect
import os
import subprocess

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "su3_oracle.c")

# (name, function whose body is mutated, old text, new text)
MUTANTS = [
    ("fwd_real_sign", "su3o_mult_nn(", "re += ar * br - ai * bi;", "re += ar * br + ai * bi;"),
    ("fwd_imag_sign", "su3o_mult_nn(", "im += ar * bi + ai * br;", "im += ar * bi - ai * br;"),
    ("fwd_b_transposed", "su3o_mult_nn(", "b[bx(j, m, l)]", "b[bx(j, l, m)]"),
    ("fwd_a_transposed", "su3o_mult_nn(", "a[ix(i, j, k, m)]", "a[ix(i, j, m, k)]"),
    ("fwd_wrong_link", "su3o_mult_nn(", "b[bx(j, m, l)]", "b[bx((j + 1) % 4, m, l)]"),
    ("fwd_dropped_term", "su3o_mult_nn(", "for (int m = 0; m < 3; ++m)", "for (int m = 0; m < 2; ++m)"),
    ("fwd_accumulate", "su3o_mult_nn(", "c[ix(i, j, k, l)] = re;", "c[ix(i, j, k, l)] += re;"),
    ("bwd_no_conj_b", "su3o_mult_nn_bwd(", "const double bi = -b[bx(j, m, l) + 1];",
     "const double bi = b[bx(j, m, l) + 1];"),
    ("bwd_no_conj_a", "su3o_mult_nn_bwd(", "const double ai = -a[ix(s, j, k, m) + 1];",
     "const double ai = a[ix(s, j, k, m) + 1];"),
    ("bwd_b_not_transposed", "su3o_mult_nn_bwd(", "const double br = b[bx(j, m, l)];",
     "const double br = b[bx(j, l, m)];"),
    ("bwd_db_dropped_k", "su3o_mult_nn_bwd(", "for (int k = 0; k < 3; ++k) {", "for (int k = 0; k < 2; ++k) {"),
    ("bwd_no_compensation", "su3o_mult_nn_bwd(", "db[q] = sum[q] + comp[q];", "db[q] = sum[q];"),
    ("recon_no_conj", "su3o_recon_row2(", "r2[2*l+1] = -xi;", "r2[2*l+1] = xi;"),
    ("recon_reversed", "su3o_recon_row2(", "const int p = (l + 1) % 3, q = (l + 2) % 3;",
     "const int q = (l + 1) % 3, p = (l + 2) % 3;"),
    ("recon32_no_conj", "recon_row2_f32(", "r2[2*l+1] = -xi;", "r2[2*l+1] = xi;"),
    ("bf16_truncate", "f32_to_bf16(", "u += 0x7fffu + ((u >> 16) & 1u);", ""),
    ("bf16_ties_away", "f32_to_bf16(", "u += 0x7fffu + ((u >> 16) & 1u);", "u += 0x8000u;"),
    ("unitarity_no_conj", "su3o_unitarity_dev(", "xi = -M[2*(3*r+p)+1];", "xi = M[2*(3*r+p)+1];"),
    ("det_sign", "su3o_det(", "cmul(M[2*l], M[2*l+1], t1r - t2r, t1i - t2i, &mr, &mi);",
     "cmul(M[2*l], M[2*l+1], t1r + t2r, t1i + t2i, &mr, &mi);"),
    ("f32_real_sign", "su3o_mult_nn_f32(", "re += ar * br - ai * bi;", "re += ar * br + ai * bi;"),
    ("soa_index_swap", "su3o_aos_to_soa(", "memcpy(D + ((int64_t)p * sites + s) * elem_bytes,",
     "memcpy(D + (s * SITE_C + p) * elem_bytes,"),
    ("pack_r12_wrong_row", "su3o_pack_r12(", "dst[o] = (float)src[ix(s, j, k, l)];",
     "dst[o] = (float)src[ix(s, j, k + 1, l)];"),
    ("na_no_conj", "su3o_mult_na(", "const double bi = -b[bx(j, l, m) + 1];",
     "const double bi = b[bx(j, l, m) + 1];"),
    ("na_not_transposed", "su3o_mult_na(", "b[bx(j, l, m)]", "b[bx(j, m, l)]"),
    ("an_no_conj", "su3o_mult_an(", "const double ai = -a[ix(i, j, m, k) + 1];",
     "const double ai = a[ix(i, j, m, k) + 1];"),
    ("an_not_transposed", "su3o_mult_an(", "a[ix(i, j, m, k)]", "a[ix(i, j, k, m)]"),
    ("r12f64_rows_swapped", "su3o_mult_nn_r12_f64(", "su3o_recon_row2(L, L + 6, L + 12);",
     "su3o_recon_row2(L + 6, L, L + 12);"),
    ("matvec_sign", "su3o_mat_vec(", "re += ar * vr - ai * vi;", "re += ar * vr + ai * vi;"),
    ("matvec_wrong_site", "su3o_mat_vec(", "v[2 * (3 * i + m)]", "v[2 * (3 * ((i + 1) % sites) + m)]"),
    ("matvec_conj_v", "su3o_mat_vec(", "const double vi = v[2 * (3 * i + m) + 1];",
     "const double vi = -v[2 * (3 * i + m) + 1];"),
    ("bwd_da_transposed", "su3o_mult_nn_bwd(", "da[ix(s, j, k, m)] = re;\n                    da[ix(s, j, k, m) + 1] = im;",
     "da[ix(s, j, m, k)] = re;\n                    da[ix(s, j, m, k) + 1] = im;"),
    ("bwd_db_a_untransposed", "su3o_mult_nn_bwd(", "const double ar = a[ix(s, j, k, m)];\n                        const double ai = -a[ix(s, j, k, m) + 1];",
     "const double ar = a[ix(s, j, m, k)];\n                        const double ai = -a[ix(s, j, m, k) + 1];"),
    ("fwd_wrong_row", "su3o_mult_nn(", "a[ix(i, j, k, m)]", "a[ix(i, j, (k + 1) % 3, m)]"),
]


def _mutate(src: str, func: str, old: str, new: str) -> str:
    start = src.index(func, src.index("\n" + "/*"))  # skip the file header
    # the function body runs from its name to the next top-level closing brace
    end = src.index("\n}\n", start)
    body = src[start:end]
    assert old in body, (func, old)
    return src[:start] + body.replace(old, new) + src[end:]


PIN_MODULES = ("test_oracle_pins.py", "test_oracle_next.py", "test_oracle_exact.py")


def _pins():
    pins = []
    for fname in PIN_MODULES:
        spec = importlib.util.spec_from_file_location(fname[:-3], os.path.join(HERE, fname))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        pins += [f for name, f in sorted(vars(mod).items())
                 if name.startswith("test_") and "O" in inspect.signature(f).parameters]
    return pins


@pytest.mark.parametrize("name,func,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, func, old, new):
    src = open(SRC).read()
    mutated = _mutate(src, func, old, new)
    assert mutated != src
    c_path = tmp_path / ("%s.c" % name)
    so_path = tmp_path / ("%s.so" % name)
    c_path.write_text(mutated)
    subprocess.run(["gcc", *oracle.CFLAGS, str(c_path), "-o", str(so_path), "-lm"], check=True)
    mutant = oracle.Oracle(oracle.load(str(so_path)))
    failed = []
    for pin in _pins():
        try:
            pin(mutant)
        except (AssertionError, ValueError, FloatingPointError):
            failed.append(pin.__name__)
            break
    assert failed, "no pin detects mutant %s" % name
