"""The C ABI on the CPU: the library loads, exports every function that
include/tmamg.h declares, its structs have the layout a C compiler gives
them, the Python mirrors agree, and the host-side argument checks answer
before any GPU work.  No compute call is made here."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tmamg.h")


@pytest.fixture(scope="module")
def tm():
    from paper_1710_06198_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_1710_06198_amd import build
        build.build(verbose=False)
    import paper_1710_06198_amd as pkg
    pkg.load()
    return pkg


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tmamg_[a-z_0-9]+)\s*\(", text)))


def declarations_with_comments():
    """(function name, the comment block that documents it): the nearest
    block comment that starts a line above the declaration, skipping other
    declarations of the same group and enum bodies."""
    lines = open(HEADER).read().splitlines()
    out = []
    for i, ln in enumerate(lines):
        m = re.match(r"^(?:const char\*|void|int|tmamg_status)\s+(tmamg_\w+)\s*\(", ln)
        if not m:
            continue
        j = i - 1
        while j >= 0:
            t = lines[j].strip()
            if t == "};":
                while j >= 0 and not lines[j].startswith(("enum", "typedef")):
                    j -= 1
            elif t.endswith("*/") and t.startswith(("/*", "*")):
                break
            j -= 1
        k = j
        while k >= 0 and not lines[k].startswith("/*"):
            k -= 1
        out.append((m.group(1), "\n".join(lines[k:j + 1])))
    return out


def test_every_call_cites_its_passage_or_says_what_it_is():
    """Each call's comment names the passage of the paper it implements
    (Sec./Eq.) or says it is plumbing, measurement or a test hook."""
    decl = declarations_with_comments()
    assert {n for n, _ in decl} == set(declared_functions())
    for name, comment in decl:
        ok = re.search(r"Sec\. \d|Eq\. \(?\d", comment) or re.search(
            r"plumbing|Plumbing|Measurement|measurement|Test hook|test hook|cannot allocate", comment)
        assert ok, (name, comment)
    solve = dict(decl)
    assert "Sec. 1.1, Eq. (1)" in solve["tmamg_solve"]
    assert "Sec. 1.2" in solve["tmamg_force"]
    assert "Sec. 2" in solve["tmamg_setup_update"]


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("tmamg_create", "tmamg_setup", "tmamg_setup_update", "tmamg_solve", "tmamg_solve_shifted",
              "tmamg_force", "tmamg_apply", "tmamg_destroy", "tmamg_last_error", "tmamg_default_params"):
        assert n in names


def test_library_exports_every_declared_symbol(tm):
    lib = ctypes.CDLL(tm.binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", tm.binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (tmamg_\w+)", out))
    assert set(declared_functions()) <= exported


LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "tmamg.h"
#define F(T, f) printf(#T " " #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("tmamg_lattice size %zu\n", sizeof(tmamg_lattice));
  printf("tmamg_params size %zu\n", sizeof(tmamg_params));
  printf("tmamg_info size %zu\n", sizeof(tmamg_info));
  printf("tmamg_allocator size %zu\n", sizeof(tmamg_allocator));
  F(tmamg_allocator, alloc) F(tmamg_allocator, free) F(tmamg_allocator, user)
  F(tmamg_lattice, dims) F(tmamg_lattice, t_antiperiodic)
  F(tmamg_params, nlevels) F(tmamg_params, agg) F(tmamg_params, nv) F(tmamg_params, setup_iters)
  F(tmamg_params, init_smooth) F(tmamg_params, sap_block1) F(tmamg_params, sap_sweeps) F(tmamg_params, mr_steps)
  F(tmamg_params, l2_iters) F(tmamg_params, l2_tol) F(tmamg_params, coarsest_iters) F(tmamg_params, coarsest_tol)
  F(tmamg_params, restart) F(tmamg_params, max_iter) F(tmamg_params, precision) F(tmamg_params, storage)
  F(tmamg_params, inner_tol) F(tmamg_params, seed) F(tmamg_params, use_graph)
  F(tmamg_params, nd_coarse_coupling)
  F(tmamg_params, setup_chunk)
  F(tmamg_params, keep_test_vectors)
  F(tmamg_info, status) F(tmamg_info, outer_iters) F(tmamg_info, cycles) F(tmamg_info, true_rel_resid)
  F(tmamg_info, t_setup_s) F(tmamg_info, t_solve_s) F(tmamg_info, l2_iters_total)
  F(tmamg_info, coarsest_iters_total)
  printf("enum %d %d %d %d %d %d %d\n", TMAMG_OK, TMAMG_NOT_CONVERGED, TMAMG_EINVAL, TMAMG_ENOMEM, TMAMG_EHIP,
         TMAMG_ENUMERIC, TMAMG_ESTATE);
  printf("prec %d %d store %d %d %d %d\n", TMAMG_FP64, TMAMG_MIXED, TMAMG_STORE_FP64, TMAMG_STORE_FP32,
         TMAMG_STORE_BF16, TMAMG_STORE_FP16);
  printf("ops %d %d %d %d %d %d %d %d\n", TMAMG_OP_D64, TMAMG_OP_D32, TMAMG_OP_PROLONG, TMAMG_OP_RESTRICT,
         TMAMG_OP_DC, TMAMG_OP_SAP, TMAMG_OP_PREC, TMAMG_OP_COARSEST);
  printf("eo %d %d %d %d %d %d\n", TMAMG_OP_SCHUR64, TMAMG_OP_SCHUR32, TMAMG_OP_DDAG64, TMAMG_OP_DDAG32,
         TMAMG_OP_DCND, TMAMG_OP_SAPND);
  printf("tune %d %d %d %d %d\n", TMAMG_TUNE_COARSE_APPLY, TMAMG_TUNE_SAP1, TMAMG_TUNE_RESTRICT0,
         TMAMG_TUNE_PROLONG0, TMAMG_TUNE_SAP0);
  return 0;
}
"""


def test_struct_layout_matches_c_compiler(tm, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines()
    b = tm.binding
    classes = {"tmamg_lattice": b.Lattice, "tmamg_params": b.Params, "tmamg_info": b.Info,
               "tmamg_allocator": b.Allocator}
    for ln in lines:
        parts = ln.split()
        if parts[0] in classes and parts[1] == "size":
            assert ctypes.sizeof(classes[parts[0]]) == int(parts[2]), ln
        elif parts[0] in classes:
            assert getattr(classes[parts[0]], parts[1]).offset == int(parts[2]), ln
        elif parts[0] == "enum":
            assert [int(v) for v in parts[1:]] == [0, 1, -1, -2, -3, -4, -5]
        elif parts[0] == "prec":
            assert (int(parts[1]), int(parts[2])) == (b.FP64, b.MIXED)
            assert [int(v) for v in parts[4:]] == [b.STORE_FP64, b.STORE_FP32, b.STORE_BF16, b.STORE_FP16]
        elif parts[0] == "ops":
            assert [int(v) for v in parts[1:]] == [b.OP_D64, b.OP_D32, b.OP_PROLONG, b.OP_RESTRICT, b.OP_DC,
                                                   b.OP_SAP, b.OP_PREC, b.OP_COARSEST]
        elif parts[0] == "eo":
            assert [int(v) for v in parts[1:]] == [b.OP_SCHUR64, b.OP_SCHUR32, b.OP_DDAG64, b.OP_DDAG32,
                                                   b.OP_DCND, b.OP_SAPND]
        elif parts[0] == "tune":
            assert [int(v) for v in parts[1:]] == [b.TUNE_COARSE_APPLY, b.TUNE_SAP1, b.TUNE_RESTRICT0,
                                                   b.TUNE_PROLONG0, b.TUNE_SAP0]


def test_default_params(tm):
    p = tm.default_params()
    assert p.nlevels == 2 and list(p.agg[0]) == [4, 4, 4, 4] and p.nv[0] == 12
    assert p.setup_iters == 3 and p.sap_sweeps[0] == 4 and p.mr_steps == 4 and p.restart == 30
    assert p.precision == tm.FP64
    q = tm.default_params(nlevels=3, agg=((4, 4, 4, 4), (2, 2, 2, 2)), nv=(24, 32), sap_block1=(3, 3, 3, 3))
    assert q.nlevels == 3 and list(q.agg[1]) == [2, 2, 2, 2] and list(q.nv) == [24, 32]
    assert list(q.sap_block1) == [3, 3, 3, 3]


def _create(tm, dims, **kw):
    b = tm.binding
    lat = b.Lattice()
    for m in range(4):
        lat.dims[m] = dims[m]
    lat.t_antiperiodic = 1
    p = tm.default_params(**kw)
    h = ctypes.c_void_p()
    st = b.load().tmamg_create(ctypes.byref(h), ctypes.byref(lat), ctypes.byref(p), None, None)
    msg = b.load().tmamg_last_error()
    return st, h, msg.decode() if isinstance(msg, bytes) else str(msg)


@pytest.mark.parametrize("dims,kw,needle", [
    ((6, 8, 8, 8), {}, "multiples of the first aggregate"),
    ((8, 8, 8, 8), {"nlevels": 4}, "nlevels"),
    ((8, 8, 8, 8), {"restart": 0}, "restart"),
    ((8, 8, 8, 8), {"precision": 1, "storage": 0}, "mixed precision"),
    ((12, 8, 8, 8), {}, "even number of fine blocks"),
    ((8, 8, 8, 8), {"agg": ((2, 2, 2, 2), (1, 1, 1, 1))}, "64, 128, 192 or 256"),
    ((16, 16, 16, 16), {"nlevels": 3, "agg": ((4, 4, 4, 4), (3, 2, 2, 2))}, "second aggregate"),
])
def test_create_rejects_bad_parameters(tm, dims, kw, needle):
    st, h, msg = _create(tm, dims, **kw)
    assert st == -1, (st, msg)
    assert not h.value
    assert needle in msg


def test_null_arguments(tm):
    lib = tm.binding.load()
    assert lib.tmamg_create(None, None, None, None, None) == -1
    assert lib.tmamg_default_params(None) == -1
    assert lib.tmamg_solve(None, None, None, 1, None, 1e-10, None) == -1
    lib.tmamg_destroy(None)   # no-op


def test_missing_library_fails_loudly(tm):
    b = tm.binding
    saved = b._lib
    try:
        b._lib = None
        with pytest.raises(RuntimeError, match="not built"):
            b.load(os.path.join(ROOT, "no_such_dir", "libtmamg.so"))
    finally:
        b._lib = saved


def test_variant_table_round_trip(tm, tmp_path):
    """The kernel variant table is host logic: set, read, remove, and its
    JSON file written and read back; malformed files and bad arguments are
    rejected without changing the table."""
    tm.tune_clear()
    try:
        assert tm.tune_entries() == 0
        assert tm.tune_get(tm.TUNE_COARSE_APPLY, 48, 2592, 16) == -1
        tm.tune_set(tm.TUNE_COARSE_APPLY, 48, 2592, 16, 1)
        tm.tune_set(tm.TUNE_SAP1, 48, 2592, 1, 0)
        tm.tune_set(tm.TUNE_SAP0, 256, 663552, 24, 1)
        tm.tune_set(tm.TUNE_RESTRICT0, 24, 663552, 24, 1)
        tm.tune_set(tm.TUNE_PROLONG0, 24, 663552, 1, 0)
        assert tm.tune_entries() == 5
        assert tm.tune_get(tm.TUNE_COARSE_APPLY, 48, 2592, 16) == 1
        assert tm.tune_get(tm.TUNE_COARSE_APPLY, 48, 2592, 15) == -1
        assert tm.tune_get(tm.TUNE_SAP1, 48, 2592, 1) == 0
        path = tmp_path / "tune.json"
        tm.tune_save(str(path))
        text = path.read_text()
        assert '"tmamg-tune-1"' in text and text.count('"family"') == 5
        tm.tune_clear()
        assert tm.tune_entries() == 0
        assert tm.tune_load(str(path)) == 5
        assert tm.tune_get(tm.TUNE_SAP0, 256, 663552, 24) == 1
        assert tm.tune_get(tm.TUNE_RESTRICT0, 24, 663552, 24) == 1
        assert tm.tune_get(tm.TUNE_PROLONG0, 24, 663552, 1) == 0
        tm.tune_set(tm.TUNE_SAP0, 256, 663552, 24, -1)   # removes the entry
        assert tm.tune_get(tm.TUNE_SAP0, 256, 663552, 24) == -1 and tm.tune_entries() == 4
        bad = tmp_path / "bad.json"
        bad.write_text(text.replace('"sap1"', '"no_such_family"'))
        with pytest.raises(tm.TmamgError, match="malformed"):
            tm.tune_load(str(bad))
        bad.write_text(text.replace("[48, 2592, 16]", "[48, 2592]"))
        with pytest.raises(tm.TmamgError, match="malformed"):
            tm.tune_load(str(bad))
        with pytest.raises(tm.TmamgError, match="malformed"):
            tm.tune_load(str(tmp_path / "missing.json"))
        assert tm.tune_entries() == 4
        with pytest.raises(tm.TmamgError, match="family"):
            tm.tune_set(7, 1, 1, 1, 0)
        tm.tune_set(tm.TUNE_SAP1, 48, 8192, 12, 2)   # the level-1 SAP has a third variant
        assert tm.tune_get(tm.TUNE_SAP1, 48, 8192, 12) == 2
        tm.tune_set(tm.TUNE_SAP1, 48, 8192, 12, -1)
        tm.tune_set(tm.TUNE_SAP1, 48, 8192, 12, 3)   # and a fourth (one workgroup per SAP block)
        assert tm.tune_get(tm.TUNE_SAP1, 48, 8192, 12) == 3
        tm.tune_set(tm.TUNE_SAP1, 48, 8192, 12, -1)
        with pytest.raises(tm.TmamgError, match="variant"):
            tm.tune_set(tm.TUNE_SAP1, 1, 1, 1, 4)
        with pytest.raises(tm.TmamgError, match="variant"):
            tm.tune_set(tm.TUNE_COARSE_APPLY, 1, 1, 1, 2)
        assert tm.binding.load().tmamg_autotune(None, None, 0, 1, None) == -1
    finally:
        tm.tune_clear()


def test_autograd_function_wiring(tm):
    """FermionAction's host logic with a stand-in solver on the CPU: the first
    call sets up, later calls update the setup, the gradient is the library's
    link gradient scaled by the incoming gradient, and a gradient after the
    links changed is refused."""
    import torch

    class Info:
        status = 0

        def as_dict(self):
            return {}

    class Standin:
        links_version = 0

        def __init__(self):
            self.calls = []

        def setup(self, U, kappa, csw, mu):
            self.calls.append("setup")
            self.links_version += 1

        def setup_update(self, U, iters):
            self.calls.append(("update", iters))
            self.links_version += 1

        def force(self, phi, F, tol):
            F.fill_(0.25j)
            return 3.5, Info()

        def force_link_gradient(self, F, G, scale):
            G.copy_(2 * scale * F)

    s = Standin()
    U = torch.zeros((4, 2, 2, 2, 2, 3, 3), dtype=torch.complex128, requires_grad=True)
    phi = torch.zeros((1, 2, 2, 2, 2, 4, 3), dtype=torch.complex128)
    S = tm.fermion_action(U, phi, s, 0.13, 1.0, 0.01)
    assert float(S.detach()) == 3.5 and s.calls == ["setup"]
    (3 * S).backward()
    assert torch.allclose(U.grad, torch.full_like(U.grad, 1.5j))
    S2 = tm.fermion_action(U, phi, s, 0.13, 1.0, 0.01, 1e-12, 2)
    assert s.calls == ["setup", ("update", 2)]
    s.setup(None, 0, 0, 0)   # links move before the gradient is taken
    with pytest.raises(RuntimeError, match="links changed"):
        S2.backward()


def test_binding_rejects_mismatched_buffers(tm):
    """The binding checks every buffer before the C ABI sees its pointer:
    dtype, contiguity, element count and one twisted mass or shift per
    right-hand side (a short list would be read past its end on the host)."""
    import torch
    b = tm.binding
    s = b.Solver.__new__(b.Solver)   # no context: the checks come first
    s.dims = (4, 4, 4, 4)
    s.device = None
    s.params = tm.default_params()
    V = 256
    good = torch.zeros((2, 4, 4, 4, 4, 4, 3), dtype=torch.complex128)
    with pytest.raises(ValueError, match="complex128"):
        s.solve(good.to(torch.complex64), good)
    with pytest.raises(ValueError, match="elements"):
        s.solve(good, torch.zeros((1, 4, 4, 4, 4, 4, 3), dtype=torch.complex128))
    with pytest.raises(ValueError, match="contiguous"):
        s.solve(good, good.transpose(-1, -2))
    with pytest.raises(ValueError, match="one per right-hand side"):
        s.solve(good, good.clone(), mu_rhs=[0.1])
    with pytest.raises(ValueError, match="one per right-hand side"):
        s.solve_shifted(good, good.clone(), [0.1, 0.2, 0.3])
    with pytest.raises(ValueError, match="two flavours"):
        s.solve_nd(good[:1], good[:1], 0.1, 0.05)
    with pytest.raises(ValueError, match="elements"):
        s.setup(torch.zeros((4, V, 9), dtype=torch.complex128)[:, :-1].contiguous(), 0.13, 1.0, 0.01)
    with pytest.raises(ValueError, match="torch tensor"):
        s.force(good[:1].numpy(), torch.zeros((4, V, 9), dtype=torch.complex128))
    with pytest.raises(ValueError, match="must be on cuda"):
        b.check_field("x", good, good.numel(), torch.device("cuda", 0))
    b.check_field("x", good, good.numel(), None)   # a matching buffer passes
