"""The C-ABI library loads and exports what include/*.h declares; host-side logic (CPU only)."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import qsynth
from oracle import methods as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2605_01464_amd", "libqpinv.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(qpinv_\w+)\s*\(", text))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("qpinv_init", "qpinv_solve", "qpinv_residuals", "qpinv_finalize", "qpinv_step", "qpinv_qgemm"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_mirrors_abi_names():
    import paper_2605_01464_amd as q

    for n in declared_functions():
        assert hasattr(q, n), n


def test_strerror_and_bad_arguments_without_gpu():
    import paper_2605_01464_amd as q

    assert q.qpinv_strerror(0) == "ok"
    assert q.qpinv_strerror(q.EDIVERGED) == "iteration diverged"
    assert q.qpinv_num_tile_configs(7) == q.EINVAL
    assert q.qpinv_num_tile_configs(q.GEMM_PREC["f32"]) >= 3
    assert q.qpinv_tile_config_name(q.GEMM_PREC["f64"], 0).startswith("f64")
    used, _ = q.qpinv_controller_replay(9, 1e-6, [1.0], [1.0])
    assert used == q.EINVAL


def test_batched_configuration_table_without_gpu():
    """The batched forms the library uses without autotuning (phase-synchronous 32 x 32 x 32 tiles,
    index 5; the queue form with 64 x 64 tiles, index 2) sit where the library expects them."""
    import paper_2605_01464_amd as q

    n = q.qpinv_num_batched_configs()
    names = [q.qpinv_batched_config_name(c) for c in range(n)]
    assert names[5] == "batched_sync_f32_32x32x32_mfma16"
    assert names[2] == "batched_f32_64x64x16_mfma16"
    assert all(nm.startswith(("batched_f32_", "batched_sync_f32_", "batched_flow_f32_")) for nm in names)


def test_product_configuration_tables_without_gpu():
    """The BF16 product forms the library picks without tuning sit where it expects them: index 11, the
    staged 64 x 64 tile with 8 waves and its operand tiles loaded straight into LDS (1024 or more 64 x 64
    output tiles); 0, the direct double-buffered 64 x 64 tile (256 to 1023); 1, the single-buffered 32 x 32
    tile (fewer); split BF16: 4, 128 x 128 tiles (256 or more of them), 3, 64 x 64 tiles (fewer)."""
    import paper_2605_01464_amd as q

    gp = q.GEMM_PREC["bf16"]
    names = [q.qpinv_tile_config_name(gp, c) for c in range(q.qpinv_num_tile_configs(gp))]
    assert names[11] == "bf16_64x64x32_w2x4_mfma16x16x32_staged_lds"
    assert names[8] == "bf16_64x64x32_w2x4_mfma16x16x32_staged"
    g3 = q.GEMM_PREC["bf16x3"]
    assert [q.qpinv_tile_config_name(g3, c) for c in (3, 4)] == ["bf16x3_64x64x32_w2x4_mfma16x16x32_staged_lds",
                                                                 "bf16x3_128x128x32_w4x4_mfma32x32x16_staged_lds"]
    assert names[0] == "bf16_64x64x32_w2x2_mfma16x16x32_db_occ2"
    assert names[1] == "bf16_32x32x32_w2x2_mfma16x16x32"
    assert len(set(names)) == len(names) and all(nm.startswith("bf16_") for nm in names)
    # defaults from 1024 tiles of 64 x 64: FP32 5 (64 x 64 double-buffered), FP64 6 (64 x 128 double-buffered);
    # below that FP32 6, FP64 1
    f32 = [q.qpinv_tile_config_name(q.GEMM_PREC["f32"], c) for c in (5, 6)]
    f64 = [q.qpinv_tile_config_name(q.GEMM_PREC["f64"], c) for c in (6, 1)]
    assert f32 == ["f32_64x64x16_w2x2_mfma32_db", "f32_32x32x16_w2x2_mfma16_db"]
    assert f64 == ["f64_64x128x8_w2x4_mfma16_db", "f64_32x32x16_w2x2_mfma16"]


# ------------------------------------------------------------------ stop-rule controller (host logic)
def test_controller_dx_abs_and_rel():
    import paper_2605_01464_amd as q

    d = [1.0, 1e-3, 1e-9, 1e-12]
    x = [2.0, 2.0, 2.0, 2.0]
    used, dec = q.qpinv_controller_replay(q.STOP["dx_abs"], 1e-10, d, x)
    assert used == 4 and dec[-1] == 1
    used, dec = q.qpinv_controller_replay(q.STOP["dx_rel"], 1e-9, d, x)
    assert used == 3 and dec[2] == 1  # 1e-9 <= 1e-9 * 2


def test_controller_divergence_and_e1():
    import paper_2605_01464_amd as q

    used, dec = q.qpinv_controller_replay(q.STOP["guarded"], 1e-6, [1.0, float("nan")], [1.0, 1.0])
    assert used == 2 and dec[1] == 3
    used, dec = q.qpinv_controller_replay(q.STOP["e1_rel"], 1e-12, [1, 1, 1], [1, 1, 1], [1e-3, 1e-9, 1e-13])
    assert used == 3 and dec == [0, 0, 1]


def test_controller_guarded_rise_matches_scripted_sequence():
    import paper_2605_01464_amd as q

    # relative changes: fall, reach a floor at update 5, rise at update 6
    rel = [0.9, 0.7, 0.2, 1e-3, 1e-5, 4e-5, 1e-3]
    used, dec = q.qpinv_controller_replay(q.STOP["guarded"], 1e-8, rel, [1.0] * len(rel))
    assert used == 6
    assert dec[5] == 2
    assert dec[4] == 4  # update 5 recorded as the minimum
    # an early wiggle before d fell below half its maximum is not a rise
    rel = [0.5, 0.6, 0.55, 0.1, 0.01, 0.001]
    used, dec = q.qpinv_controller_replay(q.STOP["guarded"], 1e-8, rel, [1.0] * len(rel))
    assert used == len(rel) and 2 not in dec


def test_controller_agrees_with_oracle_stop_decision():
    """Feed the oracle's own per-update scalars (FP64 run on a rounded rank-deficient matrix whose
    relative change eventually rises) to the library controller: both stop at the same update."""
    import paper_2605_01464_amd as q

    inst = qsynth.small_spectral_instance(5, 40, 30, qsynth.geometric(20, 1.0, 1e-4))
    A = qsynth.round_f32(inst["A"])
    r = M.solve(A, "qhpi19", alpha=M.alpha_sigma(A), tol=1e-14, stop="guarded", side="left", max_iter=60)
    assert r.reason in ("rise", "tol")
    used, dec = q.qpinv_controller_replay(q.STOP["guarded"], 1e-14, r.dx, r.xn)
    assert used == r.iters
    assert dec[used - 1] == (2 if r.reason == "rise" else 1)


def test_batch_infos_convert_on_read_without_gpu():
    """BatchInfos: a sequence over the raw per-matrix records, each turned into solve's dict when read."""
    import paper_2605_01464_amd as q

    raw = (q.Info * 3)()
    for i in range(3):
        raw[i].iters = 10 + i
        raw[i].stop_reason = 0
        raw[i].reserved = -i
    infos = q.BatchInfos(raw, 3)
    assert len(infos) == 3
    assert infos[1]["iters"] == 11 and infos[1]["status"] == -1 and infos[1]["reason"] == q.REASON[0]
    assert infos[-1]["iters"] == 12
    assert [d["iters"] for d in infos] == [10, 11, 12]
    assert [d["iters"] for d in infos[1:]] == [11, 12]
    assert infos[0] is infos[0]
    with pytest.raises(IndexError):
        infos[3]


def test_split_product_configuration_table_without_gpu():
    """The three-product (split BF16) precision has its own staged configurations, default first."""
    import paper_2605_01464_amd as q

    gp = q.GEMM_PREC["bf16x3"]
    n = q.qpinv_num_tile_configs(gp)
    names = [q.qpinv_tile_config_name(gp, c) for c in range(n)]
    assert n >= 1 and all(nm.startswith("bf16x3_") and "_staged" in nm for nm in names), names
    assert q.qpinv_num_tile_configs(4) == q.EINVAL
