"""The C-ABI library loads and exports every function include/ntrupkg.h
declares; argument validation works without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ntrupkg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ntrup_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2106_08759_amd as nk
    from paper_2106_08759_amd import build
    if not os.path.exists(nk.LIB_PATH):
        build.build()
    return nk.lib()


def test_header_declares_the_api():
    names = declared_functions()
    for n in ("ntrup_batch_keygen", "ntrup_keygen_plain", "ntrup_batch_keygen_mixed", "ntrup_ctx_create",
              "ntrup_op_mul_rq", "ntrup_op_recip_rq", "ntrup_op_recip_r3", "ntrup_op_batch_inv_rq"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_params_and_errors_without_gpu(lib):
    import paper_2106_08759_amd as nk
    for p, (q, w, pkb, skb) in {653: (4621, 288, 1062, 328), 761: (4591, 286, 1237, 382),
                                857: (5167, 322, 1393, 430), 1277: (7879, 492, 2076, 640)}.items():
        prm = nk.params(p)
        assert (prm.q, prm.w, prm.pk_bytes, prm.sk_bytes) == (q, w, pkb, skb)
    assert lib.ntrup_params(760, None, None, None, None) == nk.NTRUP_EINVAL
    # null context / bad arguments are rejected before any device work
    assert lib.ntrup_batch_keygen(None, 761, bytes(32), 0, 1, 1, 1, None, None, None, None) == nk.NTRUP_EINVAL
    assert lib.ntrup_ctx_create(None, 0, 0) == nk.NTRUP_EINVAL
    # workspace needed per call: grows with n, unknown p needs none
    assert nk.workspace_bytes(761, 1) > 0
    # (a fixed part: the tree form's heap rows; per key at least the int16
    # prefix row)
    assert nk.workspace_bytes(761, 65536) - nk.workspace_bytes(761, 1) > 65535 * 2 * 761
    assert nk.workspace_bytes(760, 1) == 0
    assert lib.ntrup_strerror(nk.NTRUP_EAGAIN).decode().startswith("no invertible")


def test_persistent_timeout_code_has_a_message():
    import paper_2106_08759_amd as nk
    lib = nk.lib()
    assert nk.NTRUP_ETIME == -62
    assert "waited too long" in lib.ntrup_strerror(nk.NTRUP_ETIME).decode()
