"""The C-ABI library loads and exports every function include/lhmm.h declares
(no device work: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lhmm_\w+)\s*\(", text, flags=re.M))
    return names


def test_library_exports_every_declared_symbol():
    from paper_2512_13267_amd import _lib

    assert os.path.exists(_lib.LIB_PATH), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(_lib.LIB_PATH)
    declared = _declared()
    assert "lhmm_micro_step" in declared and "lhmm_micro_create" in declared
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_lib.EXPORTS) <= declared


def test_binding_struct_layout_matches_header():
    from paper_2512_13267_amd import _lib

    # lhmm_params: 9 doubles, uint64, three int32 (+4 padding) ; lhmm_box: 4 x 4 bytes + 9 doubles
    assert ctypes.sizeof(_lib.LhmmParams) == 9 * 8 + 8 + 3 * 4 + 4
    assert ctypes.sizeof(_lib.LhmmBox) == 16 + 72
    assert ctypes.sizeof(_lib.LhmmSphParams) == 13 * 8 + 4 * 4  # four int32
    assert ctypes.sizeof(_lib.LhmmSurParams) == 5 * 4
    assert ctypes.sizeof(_lib.LhmmMicroConfig) == 9 * 4
    assert ctypes.sizeof(_lib.LhmmHybridParams) == 10 * 4
    assert ctypes.sizeof(_lib.LhmmHybridStats) == 2 * 8 + 6 * 4
    assert _lib.LhmmBox.h0.offset == 16


def test_null_and_bad_arguments_rejected_without_gpu():
    """Argument checks run before any device call."""
    from paper_2512_13267_amd import _lib

    lib = _lib.lib()
    out = ctypes.c_void_p()
    assert lib.lhmm_micro_create(None, None, 0, None, ctypes.byref(out)) == _lib.LHMM_ERR_ARG
    p = _lib.LhmmParams(a=25, gamma=4.5, sigma=3, kBT=1, mass=1, rc=1, dt=0.01, H=30, R0=1.5, seed=1,
                        chain_len=10, precision=0, flags=0)
    boxes = (_lib.LhmmBox * 1)()
    assert lib.lhmm_micro_create(ctypes.byref(p), boxes, 0, None, ctypes.byref(out)) == _lib.LHMM_ERR_ARG
    assert b"n_boxes" in lib.lhmm_last_error()
    boxes[0].n_particles = 100
    boxes[0].n_chains = 50  # 500 beads > 100 particles
    for q, v in enumerate([5, 0, 0, 0, 5, 0, 0, 0, 5]):
        boxes[0].h0[q] = v
    assert lib.lhmm_micro_create(ctypes.byref(p), boxes, 1, None, ctypes.byref(out)) == _lib.LHMM_ERR_ARG
    boxes[0].n_chains = 2
    boxes[0].h0[2] = 1.0  # out-of-plane coupling
    assert lib.lhmm_micro_create(ctypes.byref(p), boxes, 1, None, ctypes.byref(out)) == _lib.LHMM_ERR_ARG
    boxes[0].h0[2] = 0.0
    p.dt = -1.0
    assert lib.lhmm_micro_create(ctypes.byref(p), boxes, 1, None, ctypes.byref(out)) == _lib.LHMM_ERR_ARG
    assert lib.lhmm_micro_destroy(None) == _lib.LHMM_OK
