"""Coefficient tables of the composite odd quintic filters (oracle copy).

ORACLE — test infrastructure only. Nothing in the product library imports this
module; the HIP library carries its own transcription of the same tables.

Each stage polynomial is f_t(x) = a_t x + b_t x^3 + c_t x^5, d_t = 5 for every t
(Section 3.3, "Explicit formulations").

* ``F_STAR_SINGLE`` / ``F_TILDE_SINGLE``: Table 1, the single-precision setting,
  T = 10 (Stage-I minimax sign composite, and its Stage-II refinement).
* ``F_STAR_HALF`` / ``F_TILDE_HALF``: Table 2, the half-precision setting, T = 7.

The printed e_float of each table (Tables 1 and 2, bottom row) is kept in
``PRINTED_EFLOAT``.

Per-stage stability rescale (Section 3.4, "Numerical instability"): half
precision multiplies the iterate by 1/1.01 after every stage, single precision
by 1/1.001 after each of the first eight. The paper does not say whether the
half-precision rescale also follows the last stage. Read literally it would
leave sign(x) ~ 1/1.01 at the end and cap the ReLU error near 5e-3, which the
paper's own median half-precision errors (about 4e-4) rule out; this oracle
therefore rescales after stages 1..T-1 only in half precision (and after 1..8
in single precision, as stated).
"""
from __future__ import annotations

import numpy as np

# --- Table 1: single precision, T = 10 --------------------------------------
_F_STAR_SINGLE = [
    ("8.5098853026", "-25.2643041908", "18.7535678997"),
    ("4.2495734789", "-3.1549764881", "0.5858847825"),
    ("4.2251221908", "-3.1380444351", "0.5839534551"),
    ("4.1248386870", "-3.0683324528", "0.5760029536"),
    ("3.7580103358", "-2.8092738924", "0.5464842066"),
    ("2.8561775413", "-2.1340562332", "0.4701107692"),
    ("2.0206004158", "-1.4037211505", "0.3906738969"),
    ("1.8758751005", "-1.2509719905", "0.3750972123"),
    ("1.8750000000", "-1.2500000000", "0.3750000000"),
    ("1.8750000000", "-1.2500000000", "0.3750000000"),
]
_F_TILDE_SINGLE = [
    ("8.3119043343", "-23.0739115930", "16.4664144722"),
    ("4.1439360087", "-2.9176674704", "0.5246212487"),
    ("4.0257813209", "-2.9025002398", "0.5334261214"),
    ("3.5118574347", "-2.5740236523", "0.5050097282"),
    ("2.4398158400", "-1.7586675341", "0.4191290613"),
    ("1.9779835097", "-1.3337358510", "0.3772169049"),
    ("1.9559726949", "-1.3091355170", "0.3746734515"),
    ("1.9282822454", "-1.2823649693", "0.3704626545"),
    ("1.9220135179", "-1.2812524618", "0.3707011753"),
    ("1.8942192942", "-1.2613293407", "0.3676616051"),
]

# --- Table 2: half precision, T = 7 ------------------------------------------
_F_STAR_HALF = [
    ("8.4703288038", "-25.1080747067", "18.6292755991"),
    ("4.1828341833", "-3.1087011099", "0.5806066814"),
    ("3.9618572790", "-2.9540637464", "0.5629761180"),
    ("3.2865862170", "-2.4647201345", "0.5073576939"),
    ("2.2737499945", "-1.6446603679", "0.4161909275"),
    ("1.8887161973", "-1.2651572253", "0.3765189256"),
    ("1.8750008858", "-1.2500009843", "0.3750000984"),
]
_F_TILDE_HALF = [
    ("8.2885332412", "-22.5927099246", "15.8201383114"),
    ("4.1666196466", "-2.9679004036", "0.5307623217"),
    ("4.0611848147", "-2.9698947955", "0.5492133813"),
    ("3.6678301399", "-2.7561018955", "0.5421513305"),
    ("2.7632556383", "-2.0607754898", "0.4695405857"),
    ("2.0527445797", "-1.4345145882", "0.4070669182"),
    ("1.8804816691", "-1.2583997294", "0.3779501813"),
]


def _arr(rows):
    return np.array([[float(v) for v in r] for r in rows], dtype=np.float64)


F_STAR_SINGLE = _arr(_F_STAR_SINGLE)
F_TILDE_SINGLE = _arr(_F_TILDE_SINGLE)
F_STAR_HALF = _arr(_F_STAR_HALF)
F_TILDE_HALF = _arr(_F_TILDE_HALF)

TABLES = {
    "f_star_single": F_STAR_SINGLE,
    "f_tilde_single": F_TILDE_SINGLE,
    "f_star_half": F_STAR_HALF,
    "f_tilde_half": F_TILDE_HALF,
}

# Bottom row of Tables 1 and 2.
PRINTED_EFLOAT = {
    "f_star_single": 1.1092e-5,
    "f_tilde_single": 8.7023e-6,
    "f_star_half": 7.2868e-5,
    "f_tilde_half": 4.9233e-5,
}


def rescale_vector(name: str) -> np.ndarray:
    """Per-stage factor s_t applied after stage t (Section 3.4)."""
    tab = TABLES[name]
    T = tab.shape[0]
    s = np.ones(T, dtype=np.float64)
    if name.endswith("_half"):
        s[: T - 1] = 1.0 / 1.01
    else:
        s[: min(8, T)] = 1.0 / 1.001
    return s


def runtime_table(name: str) -> np.ndarray:
    """(a, b, c) rows with the stage rescale folded in: s_t * f_t."""
    return TABLES[name] * rescale_vector(name)[:, None]


# The refined tables are the ones the run-time projection uses (Section 4:
# single precision evaluates the refined single table, half precision the
# refined half table).
MODE_TABLE = {
    "fp32": "f_tilde_single",
    "fp16": "f_tilde_half",
    "bf16": "f_tilde_half",
    "fp16_split": "f_tilde_half",
    "fp32_emu": "f_tilde_single",
    "fp8_fp16_split": "f_tilde_half",
    "fp8_bf16_split": "f_tilde_half",
}
