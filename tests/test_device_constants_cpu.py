"""Constants the device code carries, checked on the CPU against their
definitions: the table of 2^(j/64), j = 0..63, that the double-precision
exponential kernels read (Tang's table-driven e^x), and the split of ln 2
its argument reduction uses."""
import os
import re
from decimal import Decimal, getcontext

HEADER = os.path.join(os.path.dirname(__file__), "..", "paper_2508_05958_amd", "csrc", "htlr_device.h")


def _text():
    with open(HEADER) as fh:
        return fh.read()


def test_exp2_fraction_table_is_correctly_rounded():
    src = _text()
    body = re.search(r"kExp2Frac64\[64\]\s*=\s*\{([^}]*)\}", src).group(1)
    vals = [float.fromhex(t.strip()) for t in body.split(",") if t.strip()]
    assert len(vals) == 64
    getcontext().prec = 60
    for j, v in enumerate(vals):
        exact = Decimal(2) ** (Decimal(j) / Decimal(64))
        # the double nearest the exact value: no other double is closer
        err = abs(Decimal(v) - exact)
        ulp = Decimal(2) ** (Decimal(-52))      # values lie in [1, 2)
        assert err <= ulp / 2, (j, v)


def test_ln2_split():
    src = _text()
    hi = float(re.search(r"kLn2 = ([0-9.e+-]+);", src).group(1))
    lo = float(re.search(r"kLn2Lo = ([0-9.e+-]+);", src).group(1))
    getcontext().prec = 60
    ln2 = Decimal(2).ln()
    assert Decimal(hi) == Decimal(float(ln2))              # the double nearest ln 2
    assert abs(Decimal(hi) + Decimal(lo) - ln2) < Decimal(2) ** -105
