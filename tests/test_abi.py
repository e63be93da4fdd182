"""The C-ABI library loads and exports every entry point include/lp.h
declares; sizing helpers and argument validation behave as documented
(no GPU needed: every call here fails before touching the device)."""
import ctypes as C
import os
import re

import pytest

from paper_1612_06592_amd import lp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "lp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lp_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    L = lp.lib()
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(lp.exported_symbols()) <= set(names)


def test_sizing_helpers():
    assert lp.nbytes("lp_beam_bytes", 61, 244, 32768) == 61 * 244 * 32768 * 8
    assert lp.nbytes("lp_dd_state_bytes", 7, 244) == 7 * 244 * 2048 * 8
    assert lp.nbytes("lp_dd_bytes", 7, 32, 244, 65536) == 7 * 32 * 244 * 65536 * 8
    assert lp.nbytes("lp_syn_state_bytes", 224, 244) == 224 * 244 * 16 * 8
    assert lp.nbytes("lp_cand_bytes", 2, 4096) == 2 * 4096 * 8 + 2 * 256 * 4
    assert lp.nbytes("lp_trigger_work_bytes", 1, 1, 2048) > 0
    assert lp.nbytes("lp_trigger_work_bytes", 7, 32, 65536) >= 7 * 32 * 65536 * 8
    assert lp.nbytes("lp_trigger_work_bytes", 1, 1, 0) == 0


def test_version_and_null_ctx_errors():
    L = lp.lib()
    assert b"gfx950" in L.lp_version()
    band = lp.Band(range(52, 60))
    rc = L.lp_dedisperse(None, C.byref(band.c), None, 1, None, 1, 2048,
                         None, 0, None, None)
    assert rc == lp.LP_EINVAL
    assert b"NULL" in L.lp_last_error()
    rc = L.lp_trigger(None, None, 1, 1, 2048, 0, 6.0, None, 0, None, None,
                      None, None, None, None)
    assert rc == lp.LP_EINVAL


def test_ctx_create_without_device_reports_ehip():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    rc = lp.lib().lp_ctx_create(0, C.byref(h))
    assert rc == lp.LP_EHIP and not h


def test_one_hip_runtime_per_process():
    """Loading the library maps a single HIP runtime and a single HSA
    runtime (torch's, when torch is installed), whatever was imported
    before: two copies in one process leave torch without a device."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1612_06592_amd import lp\n"
            "lp.lib()\n"
            "m = open('/proc/self/maps').read().splitlines()\n"
            "hip = {l.split()[-1] for l in m if 'libamdhip64' in l}\n"
            "hsa = {l.split()[-1] for l in m if 'libhsa-runtime64' in l}\n"
            "print(len(hip), len(hsa))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["1", "1"], out.stdout


def test_dedisperse_synthesize_sizes_and_null_arguments():
    L = lp.lib()
    assert lp.nbytes("lp_ddsyn_work_bytes", 244, 65536, 8) == 8 * 244 * 65536 * 8
    assert lp.nbytes("lp_ddsyn_work_bytes", 244, 65536, 0) == 0
    band = lp.Band(range(52, 60))
    tec = (C.c_double * 2)(0.0, 5.0)
    rc = L.lp_dedisperse_synthesize(None, C.byref(band.c), tec, 2, None, 1,
                                    2048, 0, None, None, None, 1, None, 0,
                                    None)
    assert rc == lp.LP_EINVAL
    assert b"NULL" in L.lp_last_error()


def test_binding_tec_arguments():
    """The TEC list reaches the library as contiguous doubles whatever the
    caller passes, a ctypes double array as it is; a pipeline's cached
    array follows in-place edits and replacements of its trials."""
    import numpy as np
    arr = (C.c_double * 3)(1.0, 2.0, 3.0)
    p, n = lp._tec(arr)
    assert p is arr and n == 3
    p, n = lp._tec([1.5, 2.5])
    assert n == 2 and (p[0], p[1]) == (1.5, 2.5)
    p, n = lp._tec(np.float32(7.0))
    assert n == 1 and p[0] == 7.0
    p, n = lp._tec(np.arange(8.0)[::2])        # strided: copied
    assert n == 4 and [p[i] for i in range(4)] == [0.0, 2.0, 4.0, 6.0]

    class Holder:
        pass
    h = Holder()
    h.tec = np.array([0.0, 1.0, 2.0])
    a = lp.Pipeline._tec_arg(h)
    assert list(a) == [0.0, 1.0, 2.0]
    assert lp.Pipeline._tec_arg(h) is a         # unchanged: cached
    h.tec[1] = 5.0
    b = lp.Pipeline._tec_arg(h)
    assert list(b) == [0.0, 5.0, 2.0] and b is not a
    h.tec = np.array([3.0])
    assert list(lp.Pipeline._tec_arg(h)) == [3.0]


def test_pipeline_candidate_slots_validated_before_allocation():
    """cand_slots other than 1 or 2 is refused before any device buffer is
    made (no GPU needed to reach the check)."""
    import numpy as np
    band = lp.Band(np.arange(52, 60))
    dirs = lp.Dirs(np.array([[0.0, 1.0]]))
    arr = lp.Array(np.zeros((2, 3)), 2)
    for bad in (0, 3):
        with pytest.raises(ValueError):
            lp.Pipeline(None, arr, band, dirs, [0.0], 2048, cand_slots=bad)
