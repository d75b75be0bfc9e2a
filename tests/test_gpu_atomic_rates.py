"""pml_pic_atomic_rates, the measurement aid behind the choice of an FP64 LDS box in the push
kernels: the four rates come back finite and positive through the C ABI, and a NULL output is
rejected with PML_PIC_E_INVALID_ARG."""
import ctypes as C
import math

import pytest

from gpu_helpers import say
from paper_2201_09084_amd import binding as B

pytestmark = pytest.mark.gpu


def test_atomic_rates_are_positive():
    r = B.atomic_rates()
    say("atomic lane adds per second", {k: "%.3g" % v for k, v in r.items()})
    assert set(r) == {"lds_f64", "lds_f32", "global_f32", "global_f64"}
    assert all(math.isfinite(v) and v > 0 for v in r.values())


def test_atomic_rates_null_output():
    assert B.load_library().pml_pic_atomic_rates(C.POINTER(C.c_double)()) == B.PML_PIC_E_INVALID_ARG
