"""Every long numeric literal in the HIP sources against the closed form it stands for.

A mistyped transcendental constant is a systematic error that column-level
product tolerances can miss (a Matern-5/2 coefficient 1.6e-5 low once passed
the product bar and showed only in FP64 solve residuals).  Each literal with
nine or more significant digits under csrc/ must equal one of the closed
forms below to the digits written; a new constant needs its definition here.
"""

import math
import os
import re

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2605_17898_amd", "csrc")

CLOSED_FORMS = {
    "pi": math.pi,
    "2 pi": 2.0 * math.pi,
    "ln 2": math.log(2.0),
    "log2 e": 1.0 / math.log(2.0),
    "ln(2)^2 / 3 (Matern-5/2 polynomial in the log2-scaled distance)": math.log(2.0) ** 2 / 3.0,
    "binary64 epsilon 2^-52": 2.0 ** -52,
}

LITERAL = re.compile(r"(?<![\w.])(\d+\.\d+)([eE][-+]?\d+)?f?(?![\w.])")


def _long_literals():
    found = []
    for name in sorted(os.listdir(CSRC)):
        if not name.endswith((".hip", ".hpp", ".cpp", ".h")):
            continue
        with open(os.path.join(CSRC, name)) as f:
            for lineno, line in enumerate(f, 1):
                code = line.split("//", 1)[0]
                for m in LITERAL.finditer(code):
                    digits = m.group(1).replace(".", "").lstrip("0")
                    if len(digits) >= 9:
                        found.append((name, lineno, m.group(1) + (m.group(2) or "")))
    return found


def test_sources_have_long_literals():
    # the scan itself works (the sources do hold such constants)
    assert len(_long_literals()) >= 5


@pytest.mark.parametrize("name,lineno,text", _long_literals())
def test_literal_is_a_closed_form(name, lineno, text):
    value = float(text)
    written = len(re.split("[eE]", text)[0].replace(".", "").lstrip("0"))
    # agreement to the digits written, at most what a double holds
    tol = 10.0 ** (-min(written, 16) + 1)
    best = min(CLOSED_FORMS.items(), key=lambda kv: abs(kv[1] - value) / kv[1])
    assert abs(best[1] - value) / best[1] <= tol, (name, lineno, text, best)
