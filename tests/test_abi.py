"""The C-ABI library loads and exports every function that include/*.h declares; host-side
argument validation rejects bad inputs before touching the GPU (no GPU needed)."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for hdr in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(hdr).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(nmfa_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("nmfa_create", "nmfa_anneal", "nmfa_energies", "nmfa_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1806_08422_amd import nmfa

    lib = ctypes.CDLL(nmfa.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(nmfa.EXPORTS) <= set(_declared())


def _create_rc(J, h=None, **kw):
    from paper_1806_08422_amd import nmfa

    with pytest.raises(nmfa.NmfaError) as ei:
        nmfa.Solver(J, h, **kw)
    return ei.value.code, str(ei.value)


def test_rejects_asymmetric_couplings():
    J = np.array([[0.0, 1.0], [2.0, 0.0]])
    code, msg = _create_rc(J)
    assert code == -1 and "symmetric" in msg


def test_rejects_diagonal_and_nan():
    assert _create_rc(np.eye(3))[0] == -1
    J = np.zeros((3, 3))
    J[0, 1] = J[1, 0] = np.nan
    assert _create_rc(J)[0] == -1
    assert _create_rc(np.zeros((3, 3)), np.array([0.0, np.inf, 0.0]))[0] == -1


def test_validation_names_the_first_offender_at_large_n():
    # n = 600 runs the checks on several host threads; the first violation in row-major order is
    # reported all the same
    import instances

    J = instances.sk(600, 3).J.copy()
    J[300, 450] += 1.0   # pair (300, 450) asymmetric
    J[400, 20] += 2.0    # pair (20, 400) asymmetric: first in row-major order
    code, msg = _create_rc(J)
    assert code == -1 and "symmetric at (20, 400)" in msg
    J = instances.sk(600, 3).J.copy()
    J[100, 7] = J[7, 100] = np.nan
    J[50, 590] = J[590, 50] = np.inf
    code, msg = _create_rc(J)
    assert code == -1 and "J[7][100] is not finite" in msg  # (7, 100) precedes (50, 590)


def test_rejects_bad_parameters_and_schedules():
    J = np.zeros((4, 4))
    assert _create_rc(J, alpha=0.0)[0] == -1
    assert _create_rc(J, alpha=1.5)[0] == -1
    assert _create_rc(J, sigma=-0.1)[0] == -1
    assert _create_rc(J, knots=[(0.0, 1.0), (1.0, -2.0)])[0] == -1
    assert _create_rc(J, knots=[(0.0, 1.0), (0.5, 0.5), (0.4, 0.2), (1.0, 0.1)])[0] == -1
    assert _create_rc(J, knots=[(0.1, 1.0), (1.0, 0.5)])[0] == -1
    assert _create_rc(J, precision=7)[0] == -1
    # explicit temperatures (the schedule given point by point) must be finite and positive
    assert _create_rc(J, temperatures=[1.0, 0.0, 0.5])[0] == -1
    assert _create_rc(J, temperatures=[1.0, np.nan])[0] == -1
    assert _create_rc(J, temperatures=[2.0, -1.0])[0] == -1


def test_params_struct_matches_the_header():
    """The binding's nmfa_params has the size the library expects (struct_size check)."""
    from paper_1806_08422_amd import nmfa

    p = nmfa.Params()
    nmfa.lib.nmfa_params_default(ctypes.byref(p))
    assert p.struct_size == ctypes.sizeof(nmfa.Params)
    assert p.n_T_explicit == 0 and not p.T_explicit
    assert p.alpha == 0.15 and p.sigma == 0.15


def test_server_rejects_bad_parameters():
    from paper_1806_08422_amd import nmfa

    with pytest.raises(nmfa.NmfaError) as ei:
        nmfa.Server(max_active=0)
    assert ei.value.code == -1
    with pytest.raises(nmfa.NmfaError):
        nmfa.Server(chunk_iters=0)
    with pytest.raises(nmfa.NmfaError):
        nmfa.Server(precision=9)
