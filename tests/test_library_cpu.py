"""Host-side checks of the C-ABI library (no GPU calls).

The library must load, export every function include/vgtb.h declares, size
its arena, and reject inconsistent system descriptions before touching a
device.
"""
import dataclasses
import os
import re

import numpy as np
import pytest

import vgtb_synth as vs

pkg = pytest.importorskip("paper_2308_09782_amd")


def _lib():
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libvgtb.so not built")
    return pkg.load_library()


def test_header_symbols_exported(repo_root):
    lib = _lib()
    header = open(os.path.join(repo_root, "include", "vgtb.h")).read()
    declared = set(re.findall(r"^\s*(?:vgtb_status|int64_t|int32_t|const char \*|void)\s*\*?\s*(vgtb_\w+)\s*\(",
                              header, flags=re.M))
    assert declared == set(pkg.EXPORTED), declared ^ set(pkg.EXPORTED)
    for name in declared:
        assert getattr(lib, name) is not None


def test_workspace_size_scales():
    _lib()
    opts = pkg.make_options(0.2)
    small = pkg.vgtb_workspace_size(vs.config_system("si8_k64"), opts)
    mid = pkg.vgtb_workspace_size(vs.config_system("asi64_k8_scc"), opts)
    n1, n2 = 32, 256
    assert small >= 5 * 16 * n1 * n1 * 64
    assert mid >= 5 * 16 * n2 * n2 * 8
    assert pkg.vgtb_workspace_size(vs.config_system("asi64_k8_scc"), pkg.make_options(0.2, history_capacity=10)) < mid


def _expect_inval(sysm, opts=None, match=None):
    opts = opts or pkg.make_options(0.2)
    with pytest.raises(pkg.VgtbError) as ei:
        pkg.vgtb_workspace_size(sysm, opts)
    assert ei.value.status == 1
    if match:
        assert match in str(ei.value)


def test_rejects_missing_hermitian_partner():
    _lib()
    s = vs.config_system("si8_k64")
    keep = np.ones(s.n_blocks, bool)
    keep[np.nonzero(np.linalg.norm(s.blk_d, axis=1) > 0)[0][0]] = False
    bad = dataclasses.replace(s, blk_i=s.blk_i[keep], blk_j=s.blk_j[keep], blk_d=s.blk_d[keep],
                              blk_h0=s.blk_h0[keep], blk_s=s.blk_s[keep], blk_ds=s.blk_ds[keep])
    _expect_inval(bad, match="Hermitian partner")


def test_rejects_non_transposed_partner():
    _lib()
    s = vs.config_system("si8_k64")
    h0 = s.blk_h0.copy()
    b = np.nonzero(np.linalg.norm(s.blk_d, axis=1) > 0)[0][0]
    h0[b, 0, 1] += 1e-3
    _expect_inval(dataclasses.replace(s, blk_h0=h0), match="transpose")


def test_rejects_bad_weights_and_options():
    _lib()
    s = vs.config_system("si8_k64")
    _expect_inval(dataclasses.replace(s, kw=s.kw * 1.01), match="weights")
    _expect_inval(s, pkg.make_options(0.0), match="dt")
    o = pkg.make_options(0.2)
    o.history_capacity = 0
    _expect_inval(s, o)
    bad_atom = s.blk_j.copy()
    bad_atom[3] = 99
    _expect_inval(dataclasses.replace(s, blk_j=bad_atom), match="outside")


def test_rejects_asymmetric_gamma():
    _lib()
    s = vs.random_cell(5, seed=4, gamma_u=0.25)
    g = s.gamma.copy()
    g[0, 1] += 0.1
    _expect_inval(dataclasses.replace(s, gamma=g), match="symmetric")


def test_product_path_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        pkg.Propagator(vs.config_system("si8_k64"), 0.2)


def test_rejects_momentum_coupling_without_gradients_and_bad_gradients():
    _lib()
    s = vs.config_system("si8_k64")
    opts = pkg.make_options(0.2, coupling="momentum")
    _expect_inval(dataclasses.replace(s, blk_ds=None), opts, match="overlap gradients")
    g = s.blk_ds.copy()
    b = np.nonzero(np.linalg.norm(s.blk_d, axis=1) > 0)[0][0]
    g[b, 0, 0, 1] += 1e-3
    _expect_inval(dataclasses.replace(s, blk_ds=g), opts, match="overlap gradient")
    bad = pkg.make_options(0.2)
    bad.coupling = 7
    _expect_inval(s, bad, match="coupling")
    # the same system is accepted with either coupling
    assert pkg.vgtb_workspace_size(s, opts) > pkg.vgtb_workspace_size(s, pkg.make_options(0.2))


def test_crank_nicolson_options_validated_and_sized():
    _lib()
    s = vs.config_system("asi64_k8_scc")
    _expect_inval(s, pkg.make_options(0.2, "fp32", propagator="crank_nicolson"), match="FP64 only")
    _expect_inval(s, pkg.make_options(0.2, "bf16x3", propagator="crank_nicolson"), match="FP64 only")
    bad = pkg.make_options(0.2)
    bad.propagator = 3
    _expect_inval(s, bad, match="propagator")
    # the augmented system [S + i dt/2 H | S C] adds 2 N^2 complex per k
    lf = pkg.vgtb_workspace_size(s, pkg.make_options(0.2))
    cn = pkg.vgtb_workspace_size(s, pkg.make_options(0.2, propagator="crank_nicolson"))
    n = s.n_orb
    assert cn - lf >= 2 * 16 * n * n * s.n_k


def test_fp16_split_form_validated_and_sized():
    _lib()
    s = vs.config_system("asi64_k8_scc")
    bad = pkg.make_options(0.2)
    bad.precision = 4
    _expect_inval(s, bad, match="precision")
    _expect_inval(s, pkg.make_options(0.2, "fp16x3", propagator="crank_nicolson"), match="FP64 only")
    # the operand planes of the bf16 split less its four extra (dithered) copies
    # of the planes of S^-1 - I, plus per-k scales, their partial maxima and the
    # slots of W's maximum (under 16 KB per k-point)
    bf = pkg.vgtb_workspace_size(s, pkg.make_options(0.2, "bf16x3"))
    fp = pkg.vgtb_workspace_size(s, pkg.make_options(0.2, "fp16x3"))
    npad = -(-s.n_orb // 64) * 64
    extra_copies = 4 * (4 * npad * npad * s.n_k * 2)
    assert fp > bf - extra_copies
    assert fp - (bf - extra_copies) < 16384 * s.n_k + 4096


def test_kernel_choices_are_validated_options():
    """The dense-product tile, the sparse-product variant and row group, and
    the graph / small-path switches are per-context options; the library reads
    no environment variable."""
    _lib()
    s = vs.config_system("asi64_k8_scc")
    chain = vs.linear_chain(8)
    _expect_inval(s, pkg.make_options(0.2, tile=4), match="tile_override")        # FP64: 1-3
    _expect_inval(s, pkg.make_options(0.2, "fp16x3", tile=6), match="tile_override")
    assert pkg.vgtb_workspace_size(s, pkg.make_options(0.2, "fp16x3", tile=5)) > 0
    assert pkg.vgtb_workspace_size(s, pkg.make_options(0.2, propagator="crank_nicolson", tile=3)) > 0
    _expect_inval(s, pkg.make_options(0.2, spmm_variant=3), match="spmm_variant")
    _expect_inval(s, pkg.make_options(0.2, spmm_variant=-13), match="spmm_variant")
    _expect_inval(chain, pkg.make_options(0.2, spmm_variant=-12), match="four orbitals")
    _expect_inval(chain, pkg.make_options(0.2, spmm_variant=-2), match="four orbitals")
    _expect_inval(s, pkg.make_options(0.2, spmm_group=5), match="spmm_group")
    _expect_inval(s, pkg.make_options(0.2, spmm_variant=1, spmm_group=16), match="matrix-core")
    bad = pkg.make_options(0.2)
    bad.flags = 8
    _expect_inval(s, bad, match="flags")
    for kw in ({"spmm_variant": -4, "spmm_group": 16}, {"spmm_variant": 2, "spmm_group": 4},
               {"spmm_variant": -11}, {"spmm_variant": -14, "spmm_group": 16},
               {"graphs": False, "small_path": False}):
        assert pkg.vgtb_workspace_size(s, pkg.make_options(0.2, **kw)) > 0
    # the row-group size changes the stored neighbour lists, so it reaches the sizing
    a = pkg.vgtb_workspace_size(s, pkg.make_options(0.2, spmm_group=4))
    b = pkg.vgtb_workspace_size(s, pkg.make_options(0.2, spmm_group=16))
    assert a != b
    src = "".join(open(os.path.join(os.path.dirname(pkg.LIB_PATH), "csrc", f)).read()
                  for f in os.listdir(os.path.join(os.path.dirname(pkg.LIB_PATH), "csrc")))
    assert "getenv" not in src


def test_group_arguments_rejected_before_any_device_call():
    import ctypes
    lib = _lib()
    h = ctypes.c_void_p()
    assert lib.vgtb_group_create(None, 1, ctypes.byref(h)) == pkg.VGTB_E_INVAL
    arr = (ctypes.c_void_p * 2)(None, None)
    assert lib.vgtb_group_create(arr, 0, ctypes.byref(h)) == pkg.VGTB_E_INVAL
    assert lib.vgtb_group_create(arr, 5000, ctypes.byref(h)) == pkg.VGTB_E_INVAL
    assert lib.vgtb_group_create(arr, 2, ctypes.byref(h)) == pkg.VGTB_E_INVAL   # null contexts
    assert b"null context" in lib.vgtb_last_error(None)
    assert lib.vgtb_group_create(arr, 2, None) == pkg.VGTB_E_INVAL
    assert lib.vgtb_group_step(None, 1) == pkg.VGTB_E_INVAL
    lib.vgtb_group_destroy(None)
