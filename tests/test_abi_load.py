"""CPU-side checks of the C ABI: the library loads, exports every function
include/nwq.h declares, and rejects bad arguments before touching the
device (these calls return before any HIP runtime call)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "nwq.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nwq_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    from paper_2401_06861_amd import nwq, vqe
    lib = C.CDLL(nwq._LIB_PATH)
    names = header_functions()
    assert len(names) >= 38
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(nwq.EXPORTED) | set(vqe.EXPORTED)


def test_validation_errors_without_device():
    from paper_2401_06861_amd import nwq
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_sv_create(0)
    assert e.value.code == nwq.NWQ_ERANGE
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_sv_create(35)
    assert e.value.code == nwq.NWQ_ERANGE
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_dm_create(18)
    assert e.value.code == nwq.NWQ_ERANGE
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_apply_gate(None, "h", [0])
    assert e.value.code == nwq.NWQ_EINVAL
    assert "NULL handle" in nwq.nwq_last_error()
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_sv_create_from(None, 4)
    assert e.value.code == nwq.NWQ_EINVAL
    # the one-call VQE rejects bad shapes before touching the device
    from paper_2401_06861_amd import vqe
    jh = (C.c_double * 2)(1.0, 1.0)
    assert nwq.lib.nwq_vqe_batch(0, 1, jh, 1, None, None, None, None) == nwq.NWQ_ERANGE
    assert nwq.lib.nwq_vqe_batch(4, 0, jh, 1, None, None, None, None) == nwq.NWQ_EINVAL
    assert nwq.lib.nwq_vqe_batch(4, 1, None, 1, None, None, None, None) == nwq.NWQ_EINVAL
    assert nwq.lib.nwq_vqe_batch(4, 1, jh, 0, None, None, None, None) == nwq.NWQ_EINVAL
    assert nwq.lib.nwq_vqe_batch(4, 1, jh, 1, None, None, None, None) == nwq.NWQ_EINVAL
    nan = (C.c_double * 2)(1.0, float("nan"))
    assert nwq.lib.nwq_vqe_batch(4, 1, nan, 1, None, None, None, None) == nwq.NWQ_EINVAL
    assert vqe.lib.nwq_vqe_batch_release() == nwq.NWQ_OK
    # the allocation-free sampler rejects sizes beyond its scratch before any launch
    assert nwq.lib.nwq_sample_noalloc(21, None, None, 0, None, None) == nwq.NWQ_ERANGE


def test_gate_table_matches_header():
    from paper_2401_06861_amd import nwq
    txt = open(os.path.join(ROOT, "include", "nwq.h")).read()
    body = txt[txt.index("enum nwq_gate"):]
    body = body[:body.index("};")]
    names = re.findall(r"NWQ_GATE_([A-Z0-9]+)", body)
    names = [x for x in names if x != "COUNT"]
    want = {"I": "id"}
    for i, nm in enumerate(names):
        assert nwq.GATES[want.get(nm, nm.lower())] == i
