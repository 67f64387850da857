"""The collision kernels' work decomposition, audited on the CPU.

libkbe exports a host-side self-check, kbe_internal_audit_tasks, that walks every task of the plan
a call would launch, the way the kernels do, and counts the staged operand blocks, weights and
streamed blocks whose address falls outside their array.  This is the regression test for the
fault in which the empty term ranges of the greater form's B_GRD class (outputs outside [m0, m1))
pulled the workgroup union below m0, so the MFMA and small-block tasks staged cotangent blocks
before the start of the array.  No GPU is used: addresses are formed from dummy bases and never
dereferenced.
"""
import ctypes

import pytest

import paper_2405_08737_amd as kbe

OUT_ALL, GREATER, FORCE_GENERIC = 0xF, 0x400, 0x100
OUT_IR_IL = 0x3
BOTH = 0x10000  # library-internal: both forms in one call (the propagations), forward only
GREXTRA = 0x20000  # library-internal: the greater form's adjoint beyond the lesser form's
SAMECOT = 0x40000  # library-internal, with GREXTRA: gIR and gIL are one array (B_L, B_GRU merged)


def audit(N, nt, ntau, n, m0, m1, flags, adjoint, ldt=None):
    f = kbe.lib().kbe_internal_audit_tasks
    f.restype = ctypes.c_int64
    f.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_int64] + [ctypes.c_int32] * 3 + \
        [ctypes.c_uint32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
    checked = ctypes.c_int64(0)
    bad = f(N, nt, ntau, ldt or nt, n, m0, m1, flags, adjoint, ctypes.byref(checked))
    return bad, checked.value


CASES = [
    # N, nt, ntau, n, m0, m1
    (16, 300, 17, 299, 0, 300),
    (16, 280, 9, 279, 30, 270),   # the faulting shape: N = 16 on a partial range
    (16, 60, 8, 59, 10, 50),
    (16, 30, 6, 29, 10, 20),
    (16, 9, 3, 8, 0, 9),
    (8, 300, 20, 299, 7, 290),
    (8, 30, 6, 29, 10, 20),
    (6, 140, 30, 139, 20, 120),
    (5, 40, 0, 39, 4, 25),
    (4, 600, 40, 599, 100, 480),
    (3, 530, 60, 529, 0, 530),
    (2, 64, 64, 63, 10, 40),
    (1, 70, 4, 69, 7, 64),
    (12, 50, 7, 49, 3, 41),       # generic kernels
    (16, 300, 40, 170, 0, 171),   # row n inside the stored history
    (16, 300, 40, 299, 299, 300),
    (16, 300, 40, 299, 0, 1),
]


@pytest.mark.parametrize("N,nt,ntau,n,m0,m1", CASES)
@pytest.mark.parametrize("greater", [False, True])
@pytest.mark.parametrize("adjoint", [0, 1])
def test_every_task_stays_inside_its_arrays(N, nt, ntau, n, m0, m1, greater, adjoint):
    flags = OUT_ALL | (GREATER if greater else 0)
    bad, checked = audit(N, nt, ntau, n, m0, m1, flags, adjoint)
    assert checked > 0
    assert bad == 0, f"{bad} of {checked} addresses outside their arrays"
    if N != 16 and N > 8:
        return
    bad, checked = audit(N, nt, ntau, n, m0, m1, flags | FORCE_GENERIC, adjoint)
    assert bad == 0


@pytest.mark.parametrize("N,nt,ntau,n,m0,m1", CASES)
def test_both_forms_tasks_stay_inside_their_arrays(N, nt, ntau, n, m0, m1):
    """The propagations' call that runs the lesser and the greater form together (the greater
    form's I^< on a Sigma^> row of m1 blocks through its own class)."""
    for extra in (0, FORCE_GENERIC):
        bad, checked = audit(N, nt, ntau, n, m0, m1, OUT_ALL | BOTH | extra, 0)
        assert checked > 0
        assert bad == 0, f"{bad} of {checked} addresses outside their arrays"
        lesser = audit(N, nt, ntau, n, m0, m1, OUT_ALL | extra, 0)[1]
        greater = audit(N, nt, ntau, n, m0, m1, OUT_IR_IL | GREATER | extra, 0)[1]
        # every address of the lesser form, plus the greater form's minus its shared I^R terms
        assert lesser < checked < lesser + greater


@pytest.mark.parametrize("N,nt,ntau,n,m0,m1", CASES)
def test_greater_extra_adjoint_tasks_stay_inside_their_arrays(N, nt, ntau, n, m0, m1):
    """The propagations' adjoint of the greater form's further terms alone (library-internal),
    also with one cotangent array for I^R and I^< (two classes merged off the MFMA path)."""
    for extra in (0, FORCE_GENERIC):
        bad, checked = audit(N, nt, ntau, n, m0, m1, OUT_IR_IL | GREATER | GREXTRA | extra, 1)
        assert checked > 0
        assert bad == 0, f"{bad} of {checked} addresses outside their arrays"
        full = audit(N, nt, ntau, n, m0, m1, OUT_IR_IL | GREATER | extra, 1)[1]
        assert checked < full
        bad2, merged = audit(N, nt, ntau, n, m0, m1,
                             OUT_IR_IL | GREATER | GREXTRA | SAMECOT | extra, 1)
        assert bad2 == 0, f"{bad2} of {merged} addresses outside their arrays"
        if N == 16 and not extra:  # the MFMA path keeps the two classes
            assert merged == checked
        elif m1 > m0 + 1:  # the merged class reads B_GRU's blocks once, with B_L's
            assert 0 < merged < checked


def test_padded_row_stride():
    bad, checked = audit(16, 300, 24, 299, 0, 300, OUT_ALL, 1, ldt=30000)
    assert bad == 0 and checked > 0
