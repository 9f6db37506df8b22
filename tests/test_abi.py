"""Host-side checks of the C-ABI library (no GPU needed)."""
import os
import re

import pytest

from paper_2203_15115_amd import afdcg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "afdcg.h")).read()
    return sorted(set(re.findall(r"\b(afd_[A-Za-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_header_function():
    L = afdcg.lib()
    names = header_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    assert sorted(afdcg.EXPORTED) == names


def test_no_device_is_reported_not_faked():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(afdcg.AfdError) as ei:
        afdcg.afd_context_create(0, None)
    assert ei.value.code == afdcg.AFD_E_NO_DEVICE
    assert "device" in afdcg.lib().afd_last_error().decode()


def test_null_arguments_rejected_without_device():
    L = afdcg.lib()
    assert L.afd_mesh_create(None, None, None) in (afdcg.AFD_E_INVALID_ARG,)
    assert L.afd_solve(None, None, 1, None, None, None, None, None) == afdcg.AFD_E_INVALID_ARG
    assert L.afd_mesh_sizes(None, None, None, None, None) == afdcg.AFD_E_INVALID_ARG
    assert L.afd_mesh_solver_form(None, afdcg.AFD_FORM_LAUNCHES) == afdcg.AFD_E_INVALID_ARG
