"""The C-ABI library loads and exports every symbol its header declares; its
argument checks run on the host and reject bad calls before any GPU work
(no GPU needed)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbg.h")


def _lib():
    import paper_0910_4711_amd as P
    if not os.path.exists(P.library_path()):
        from paper_0910_4711_amd import build
        build.build()
    return P, P.load()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_calls():
    names = _declared()
    for need in ["lbg_split", "lbg_assign", "lbg_update", "lbg_distortion", "lbg_train",
                 "lbg_workspace_size", "lbg_last_error", "lbg_distortion_backward",
                 "lbg_centroid", "lbg_split_add", "lbg_params_default", "lbg_version",
                 "lbg_assign_batched", "lbg_update_batched"]:
        assert need in names


def test_library_exports_every_declared_symbol():
    _, lib = _lib()
    for name in _declared():
        assert hasattr(lib, name), name


def test_version_and_defaults():
    P, lib = _lib()
    assert b"gfx950" in lib.lbg_version()
    p = P.Params()
    lib.lbg_params_default(ct.byref(p))
    assert p.thr == 1e-3 and p.eps_split == 0.01 and p.max_iter == 1000
    assert p.split_mode == P.SPLIT_MULT and p.precision == P.FP32


FAKE = ct.c_void_p(1 << 20)  # never dereferenced: every call below fails its checks


def test_argument_checks_reject_bad_sizes():
    P, lib = _lib()
    assert lib.lbg_split(FAKE, 0, 4, 0.01, FAKE, None) == P.EINVAL
    assert b"N = 0" in lib.lbg_last_error()
    assert lib.lbg_split(FAKE, 4, 0, 0.01, FAKE, None) == P.EINVAL
    assert lib.lbg_split(FAKE, 4, 300, 0.01, FAKE, None) == P.EINVAL
    assert lib.lbg_split(FAKE, 4, 4, 1.5, ct.c_void_p((1 << 20) + 4096), None) == P.EINVAL
    assert b"eps" in lib.lbg_last_error()
    assert lib.lbg_split(FAKE, 4, 4, 0.01, FAKE, None) == P.EINVAL  # overlap
    assert b"overlap" in lib.lbg_last_error()
    assert lib.lbg_assign(FAKE, 0, 16, FAKE, 4, FAKE, None, 0, None, 0, None) == P.EINVAL
    assert lib.lbg_assign(FAKE, 10, 16, FAKE, 70000, FAKE, None, 0, None, 0, None) == P.EINVAL
    assert lib.lbg_assign(FAKE, 10, 16, FAKE, 4, FAKE, None, 7, None, 0, None) == P.EINVAL
    assert b"precision" in lib.lbg_last_error()
    assert lib.lbg_assign(None, 10, 16, FAKE, 4, FAKE, None, 0, None, 0, None) == P.EINVAL
    assert b"X is NULL" in lib.lbg_last_error()
    assert lib.lbg_assign(ct.c_void_p((1 << 20) + 2), 10, 16, FAKE, 4, FAKE, None, 0, None,
                          0, None) == P.EINVAL
    assert b"aligned" in lib.lbg_last_error()


def test_argument_checks_workspace():
    P, lib = _lib()
    need = lib.lbg_workspace_size(P.OP_UPDATE, 1000, 16, 8, 0)
    assert need > 0
    assert lib.lbg_update(FAKE, 1000, 16, FAKE, FAKE, 8, FAKE, None, FAKE, need - 1,
                          None) == P.ENOWS
    assert lib.lbg_update(FAKE, 1000, 16, FAKE, FAKE, 8, FAKE, None, None, need,
                          None) == P.EINVAL
    assert lib.lbg_update(FAKE, 1000, 16, FAKE, FAKE, 8, FAKE, None, ct.c_void_p((1 << 20) + 64),
                          need, None) == P.EINVAL
    assert b"256-byte" in lib.lbg_last_error()
    assert lib.lbg_workspace_size(P.OP_ASSIGN, 1000, 16, 8, 0) > 0
    assert lib.lbg_workspace_size(P.OP_TRAIN, 262144, 16, 256, 0) > 0


def test_train_rejects_bad_parameters():
    P, lib = _lib()
    D = ct.c_double()
    p = P.Params()
    lib.lbg_params_default(ct.byref(p))
    args = lambda N, pp: lib.lbg_train(FAKE, 100, 4, N, pp, FAKE, FAKE, ct.byref(D), None,
                                       FAKE, 1 << 30, None)
    assert args(6, ct.byref(p)) == P.EINVAL
    assert b"power of two" in lib.lbg_last_error()
    p.thr = -1.0
    assert args(8, ct.byref(p)) == P.EINVAL
    lib.lbg_params_default(ct.byref(p))
    p.eps_split = 0.0
    assert args(8, ct.byref(p)) == P.EINVAL
    lib.lbg_params_default(ct.byref(p))
    p.split_mode = 7
    assert args(8, ct.byref(p)) == P.EINVAL
    lib.lbg_params_default(ct.byref(p))
    p.C_init, p.N_init = 1 << 20, 3
    assert args(8, ct.byref(p)) == P.EINVAL
    lib.lbg_params_default(ct.byref(p))
    p.n_forced = 2
    assert args(8, ct.byref(p)) == P.EINVAL


def test_binding_refuses_cpu_tensors():
    import torch
    P, _ = _lib()
    X = torch.zeros(8, 4)
    with pytest.raises(TypeError):
        P.assign(X, X)


def test_batched_argument_checks():
    P, lib = _lib()
    inst = (P.Instance * 2)()
    for i in range(2):
        inst[i].X, inst[i].C_out, inst[i].idx_out = FAKE.value, FAKE.value, FAKE.value
        inst[i].M, inst[i].L, inst[i].N = 100, 16, 8
    need = lib.lbg_train_batched_workspace(inst, 2)
    assert need > 0
    call = lambda n, ws, nb, p=None: lib.lbg_train_batched(inst, n, p, None, None, None, ws, nb,
                                                           None)
    assert call(2, FAKE, need - 1) == P.ENOWS
    assert b"workspace" in lib.lbg_last_error()
    assert call(2, None, need) == P.EINVAL
    assert call(0, FAKE, need) == P.EINVAL
    inst[1].N = 6
    assert call(2, FAKE, need) == P.EINVAL
    assert b"power of two" in lib.lbg_last_error()
    inst[1].N, inst[1].L = 8, 65
    assert call(2, FAKE, need) == P.EINVAL
    inst[1].L, inst[1].N = 64, 512
    assert call(2, FAKE, need) == P.EINVAL
    assert b"LDS" in lib.lbg_last_error()
    inst[1].N = 8
    p = P.Params()
    lib.lbg_params_default(ct.byref(p))
    p.precision = P.BF16_RESCORE
    assert call(2, FAKE, need, ct.byref(p)) == P.EINVAL
    inst[1].idx_out = None
    assert call(2, FAKE, need) == P.EINVAL
    assert b"NULL" in lib.lbg_last_error()
    cfg = P.BatchConfig()
    lib.lbg_batch_config_default(ct.byref(cfg))
    assert cfg.graph == 1 and cfg.grab == 0 and cfg.grid == 0
    assert cfg.screen == 0


def test_batched_single_steps_argument_checks():
    P, lib = _lib()
    items = (P.AssignItem * 2)()
    for i in range(2):
        items[i].X, items[i].C, items[i].idx = FAKE.value, FAKE.value, FAKE.value
        items[i].M, items[i].L, items[i].N = 100, 16, 9
    need = lib.lbg_assign_batched_workspace(items, 2)
    assert need > 0 and lib.lbg_assign_batched_workspace(None, 2) == 0
    call = lambda n, ws, nb: lib.lbg_assign_batched(items, n, ws, nb, None)
    assert call(2, FAKE, need - 1) == P.ENOWS
    assert call(0, FAKE, need) == P.EINVAL
    items[1].L = 65
    assert call(2, FAKE, need) == P.EINVAL
    items[1].L, items[1].N = 64, 512
    assert call(2, FAKE, need) == P.EINVAL and b"LDS" in lib.lbg_last_error()
    items[1].N, items[1].D = 9, FAKE.value + 4  # misaligned FP64 output
    assert call(2, FAKE, need) == P.EINVAL and b"misaligned" in lib.lbg_last_error()
    items[1].D, items[1].C = None, None
    assert call(2, FAKE, need) == P.EINVAL and b"NULL" in lib.lbg_last_error()
    ups = (P.UpdateItem * 1)()
    ups[0].X, ups[0].idx, ups[0].C_old, ups[0].C_new = (FAKE.value,) * 4
    ups[0].M, ups[0].L, ups[0].N = 100, 16, 8
    need = lib.lbg_update_batched_workspace(ups, 1)
    assert need > 0
    assert lib.lbg_update_batched(ups, 1, FAKE, need - 1, None) == P.ENOWS
    ups[0].N = 0
    assert lib.lbg_update_batched(ups, 1, FAKE, need, None) == P.EINVAL
    ups[0].N, ups[0].C_new = 8, None
    assert lib.lbg_update_batched(ups, 1, FAKE, need, None) == P.EINVAL
