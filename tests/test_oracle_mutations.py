"""Planted mistakes in the oracle must be caught by its pins.

Each mutant is the oracle source with one plausible mistake (bit order, a
dropped term, a wrong sign or index, a transposed operand), built into a
temporary library on the CPU.  The pin suite must reject every mutant; the
unmodified source must pass it (checked by test_oracle_pins.py).
"""
import os
import subprocess
import sys

import pytest

import oracle
from oracle_pins import ALL_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "ccmref.c")
TESTS = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(TESTS)

MUTANTS = {
    # bitstrings written from left to right instead of right to left
    "msb_first_words": [("(uint64_t)1 << (p % 64u)", "(uint64_t)1 << (63u - p % 64u)"),
                        ("(words[p / 64u] >> (p % 64u))", "(words[p / 64u] >> (63u - p % 64u))")],
    # fields written most significant bit first (consistently on both sides)
    "msb_first_fields": [("put_bit(words, p0 + (uint64_t)t,", "put_bit(words, p0 + (uint64_t)(bits - 1 - t),"),
                         ("get_bit(words, p0 + (uint64_t)t) << t", "get_bit(words, p0 + (uint64_t)(bits - 1 - t)) << t")],
    # the header's signed flag never set
    "header_flag_unsigned": [("out[7] = (uint8_t)(m->is_signed ? 1u : 0u);", "out[7] = 0;")],
    # the header's min written as its magnitude
    "header_min_magnitude": [("put_le(out + 24, (uint64_t)m->vmin, 8);",
                              "put_le(out + 24, (uint64_t)(m->vmin < 0 ? -m->vmin : m->vmin), 8);")],
    # the column-major flag replaces the signed flag instead of joining it
    "header_cm_flag_only": [("out[7] = (uint8_t)(out[7] | 2u);", "out[7] = 2u;")],
    # the "+1" of the bitstring count dropped
    "word_count": [("/ 64u + 1u", "/ 64u")],
    # bit-length off by one
    "bitlen": [("(u >> L) != 0", "(u >> L) > 1")],
    # Eq. 1's first case returns 0 bits
    "eq1_zero": [("if (sup == 0 || sup == 1) return 1;", "if (sup == 0 || sup == 1) return (int)sup;")],
    # the sign bit left out of the signed width
    "signed_width": [("*bits = 1 + (lo > hi ? lo : hi);", "*bits = (lo > hi ? lo : hi) + (lo == hi);")],
    # sign extension by 2^(b-1) instead of 2^b
    "sign_extend": [("u = u - ((uint64_t)1 << bits);", "u = u - ((uint64_t)1 << (bits - 1));")],
    # matmul reads B transposed
    "matmul_transposed": [("(uint64_t)(k * b->cols + j)", "(uint64_t)(j * b->cols + k)")],
    # matvec drops the first column
    "matvec_first_term": [("for (int64_t j = 0; j < a->cols; j++) {\n      int64_t v",
                           "for (int64_t j = 1; j < a->cols; j++) {\n      int64_t v")],
    # add subtracts
    "add_sign": [("(__int128)get_field(a->payload, (uint64_t)e, a->bits, a->is_signed) +",
                  "(__int128)get_field(a->payload, (uint64_t)e, a->bits, a->is_signed) -")],
    # overflow bound compares with > instead of >=
    "matmul_bound": [("if (p * (unsigned __int128)(uint64_t)a->cols >= lim)",
                      "if (p * (unsigned __int128)(uint64_t)a->cols > lim)")],
    # signed flag ignored when decoding
    "decode_unsigned": [("if (is_signed && ((u >> (bits - 1)) & 1u)) {", "if (0) {")],
    # column-major stream index taken row-major
    "cm_index_rowmajor": [("return (uint64_t)(j * m->rows + i);", "return (uint64_t)(i * m->cols + j);")],
    # y = A^T x reads A transposed (a[j][i])
    "matvec_t_transposed": [("(uint64_t)(i * a->cols + j), a->bits, a->is_signed);\n      acc",
                             "(uint64_t)(j * a->rows + i), a->bits, a->is_signed);\n      acc")],
    # the method choice breaks ties towards Method 2
    "method_tie": [("out->method = out->vlb_nbits < out->sm_nbits ? 2 : 1;",
                    "out->method = out->vlb_nbits <= out->sm_nbits ? 2 : 1;")],
    # Eq. 29 without the length field's k / 64
    "eta2_model_no_k": [("return 1.0 - mean / 64.0 - (double)k / 64.0;", "return 1.0 - mean / 64.0;")],
    # Method 2: the element written before its length chunk
    "vlb_value_first": [("put_bits(m->payload, p, m->k, (uint64_t)b); /* the fixed-size length chunk */\n"
                         "    p += (uint64_t)m->k;\n"
                         "    put_bits(m->payload, p, b, (uint64_t)dense[e]); /* then the element itself */\n"
                         "    p += (uint64_t)b;",
                         "put_bits(m->payload, p, b, (uint64_t)dense[e]);\n"
                         "    p += (uint64_t)b;\n"
                         "    put_bits(m->payload, p, m->k, (uint64_t)b);\n"
                         "    p += (uint64_t)m->k;")],
    # Method 2: k taken from the largest value instead of the largest width
    "vlb_k_of_value": [("m->k = ccmref_bitlen((uint64_t)bmax);",
                        "m->k = ccmref_bitlen((uint64_t)bmax) + (hi > 1);")],
    # Method 2: the length chunk holds b - 1
    "vlb_length_minus_one": [("put_bits(m->payload, p, m->k, (uint64_t)b);",
                              "put_bits(m->payload, p, m->k, (uint64_t)(b - 1));")],
    # Method 2: no sign extension on decode
    "vlb_no_sign_extend": [("if (m->is_signed && ((u >> (b - 1)) & 1u) && b < 64)", "if (0)")],
    # Method 2: the sign bit left out of non-negative elements of a signed matrix
    "vlb_signed_width": [("b = 1 + ccmref_bitlen((uint64_t)v);", "b = ccmref_bitlen((uint64_t)v) + (v == 0);")],
    # Method 2: matvec skips the last column
    "vlb_matvec_last": [("for (int64_t j = 0; j < m->cols; j++) {\n      int64_t a = vlb_next(m, &p);",
                         "for (int64_t j = 0; j < m->cols; j++) {\n      int64_t a = vlb_next(m, &p);\n"
                         "      if (j == m->cols - 1) a = 0;")],
    # fixed point: halves rounded up instead of to even
    "fx_round_half_up": [("return fmod(fl, 2.0) == 0.0 ? fl : fl + 1.0;", "return fl + 1.0;")],
    # fixed point: one fraction bit too many
    "fx_frac_bits_off_by_one": [("*frac_bits = sig_bits - 1 - (ex - 1);",
                                 "*frac_bits = sig_bits - (ex - 1);")],
    # fixed point: dequantization scales the wrong way
    "fx_dequantize_scale_sign": [("v[i] = ldexp((double)q[i], -frac_bits);",
                                  "v[i] = ldexp((double)q[i], frac_bits);")],
    # fixed point: the overflow bound admits exactly 2^62
    "fx_overflow_bound": [("if (!(fabs(t) < 0x1p62))", "if (!(fabs(t) <= 0x1p62))")],
    # fixed point: f written at the wrong header offset
    "fx_header_offset": [("put_le(out + 48, (uint64_t)(uint16_t)(int16_t)frac_bits, 2);",
                          "put_le(out + 56, (uint64_t)(uint16_t)(int16_t)frac_bits, 2);")],
}


@pytest.fixture(scope="module")
def src():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, src, tmp_path):
    text = src
    for old, new in MUTANTS[name]:
        assert old in text, f"mutation pattern not found: {old!r}"
        text = text.replace(old, new)
    c = tmp_path / "ccmref.c"
    c.write_text(text)
    (tmp_path / "ccmref.h").write_text(open(SRC[:-1] + "h").read())
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-std=gnu11", "-O1", "-fPIC", "-shared", "-fopenmp", str(c), "-o",
                    str(so)], check=True)
    # The pins run in a child process: a mutant may also crash (e.g. by writing
    # past a payload it sized wrongly), which counts as caught.
    script = (
        "import sys; sys.path[:0] = [%r, %r]\n"
        "import oracle, oracle_pins\n"
        "mut = oracle.Oracle(%r)\n"
        "failed = []\n"
        "for pin in oracle_pins.ALL_PINS:\n"
        "    try:\n"
        "        pin(mut)\n"
        "    except Exception as e:\n"
        "        failed.append(pin.__name__)\n"
        "print('FAILED', failed)\n"
        "sys.exit(1 if failed else 0)\n"
    ) % (ROOT, TESTS, str(so))
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, f"mutant {name} passed every pin: {r.stdout}{r.stderr}"
