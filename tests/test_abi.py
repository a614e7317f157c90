"""C-ABI library on the host (no GPU calls): exports, configuration checks,
and the FP64 host basis against the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle.fcc_oracle as O
from gen import circular_array, square_array

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def fcc():
    import paper_2204_13622_amd as fcc
    fcc._lib.load()
    return fcc


def _declared_functions():
    with open(os.path.join(ROOT, "include", "fcc.h")) as fh:
        src = fh.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fcc_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(fcc):
    lib = ctypes.CDLL(fcc.library_path())
    declared = _declared_functions()
    assert len(declared) >= 13
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(fcc._lib.EXPORTS)


def test_status_strings(fcc):
    lib = fcc._lib.load()
    for code, name in fcc._lib.STATUS_NAMES.items():
        assert lib.fcc_status_string(code).decode() == name


@pytest.mark.parametrize("kw,status", [
    (dict(mic_xyz=np.zeros((1, 3))), "FCC_ERR_INVALID_ARG"),
    (dict(frame_size=500), "FCC_ERR_INVALID_ARG"),
    (dict(frame_size=8), "FCC_ERR_INVALID_ARG"),
    (dict(hop=0), "FCC_ERR_INVALID_ARG"),
    (dict(fs=-1.0), "FCC_ERR_INVALID_ARG"),
    (dict(c=0.0), "FCC_ERR_INVALID_ARG"),
    (dict(rank=10), "FCC_ERR_INVALID_ARG"),          # I = 9 for the 5 cm square
    (dict(tau_max=128), "FCC_ERR_INVALID_ARG"),      # must stay below N/4
    (dict(interp=3), "FCC_ERR_INVALID_ARG"),
    (dict(interp=4, tau_max=32), "FCC_ERR_INVALID_ARG"),   # r tau_max must stay below N/4
    (dict(alpha=0.0), "FCC_ERR_INVALID_ARG"),
    (dict(alpha=1.5), "FCC_ERR_INVALID_ARG"),
    (dict(alpha=0.1, precision="bf16"), "FCC_ERR_UNSUPPORTED"),
    (dict(alpha=0.1, method="gcc"), "FCC_ERR_UNSUPPORTED"),
    (dict(interp=4, frame_size=2048, hop=512, method="gcc"), "FCC_ERR_UNSUPPORTED"),
    (dict(mic_xyz=circular_array(33, 0.05)), "FCC_ERR_UNSUPPORTED"),
])
def test_invalid_configs(fcc, kw, status):
    args = dict(mic_xyz=square_array(0.05), fs=16000.0, frame_size=512, hop=128)
    args.update(kw)
    with pytest.raises(fcc.FccError) as ei:
        fcc.Plan(**args)
    assert ei.value.name == status


def test_ambiguous_rank_refused(fcc):
    with pytest.raises(fcc.FccError) as ei:
        fcc.Plan(circular_array(16, 0.05), 48000.0, frame_size=1024, hop=256, rank=3)
    assert ei.value.name == "FCC_ERR_BASIS_AMBIGUOUS"
    with pytest.raises(O.BasisAmbiguous):
        O.fcc_basis(1024, 14, 3)


def test_plan_query(fcc):
    p = fcc.Plan(circular_array(16, 0.05), 16000.0, frame_size=512, hop=128, rank=6)
    assert (p.M, p.P, p.N, p.F, p.tau_max, p.I, p.rank) == (16, 120, 512, 257, 5, 11, 6)
    assert (p.info.rank_sym, p.info.rank_anti) == (3, 3)
    assert p.num_frames(960000) == 7497 and p.num_frames(511) == 0 and p.num_frames(512) == 1
    assert p.info.spectrum_bytes_per_frame == 16 * 256 * 8     # packed: N/2 slots
    assert p.workspace_bytes(7497) % 256 == 0
    assert fcc.Plan(square_array(0.05), 16000.0, precision="bf16").info.spectrum_elem_bytes == 4
    assert fcc.Plan(square_array(0.05), 16000.0, precision="fp8").info.spectrum_elem_bytes == 2
    g = fcc.Plan(square_array(0.05), 16000.0, method="gcc")
    assert g.rank == g.I == 9


def test_interp_and_alpha_plans(fcc):
    # the paper's operating point: tau_max = 8, r = 2 -> I = 33 (Sec. 3 and 5)
    p = fcc.Plan(np.array([[0, 0, 0], [0.15, 0, 0]]), 16000.0, c=335.0, frame_size=512, hop=256,
                 tau_max=8, rank=8, interp=2, alpha=0.1)
    assert (p.tau_max, p.I, p.rank, p.info.interp) == (8, 33, 8, 2)
    assert abs(p.info.alpha - 0.1) < 1e-7
    assert p.info.spectrum_elem_bytes == 8
    # alpha < 1: the whole-path workspace also holds the state and the chunk carries
    assert p.workspace_bytes(100) > 100 * p.info.spectrum_bytes_per_frame
    assert p.smooth_workspace_bytes(100) > 0 and p.smooth_workspace_bytes(0) == 0
    g = fcc.Plan(circular_array(4, 0.05), 16000.0, frame_size=1024, hop=256, interp=4, method="gcc")
    assert g.I == 8 * g.tau_max + 1


def _operator(e, N):
    """Rank-D frequency-to-lag operator U S V^T rebuilt from exported tables."""
    m, F = N // 4, N // 2 + 1
    D = len(e["sigma"])
    V = np.zeros((D, F))
    f = np.arange(m)
    for k in range(D):
        v = e["p_hat"][k] / e["sigma"][k]
        V[k, f] = v[:m]
        V[k, N // 2 - f] = v[:m] if e["is_sym"][k] else -v[:m]
        V[k, m] = v[m]
    return (e["Dc"] + 1j * e["Ds"]) @ (e["sigma"][:, None] * V)


@pytest.mark.parametrize("r,tau_max,D", [(2, 8, 8), (2, 8, 16), (2, 4, 17), (4, 3, 9), (2, 8, 33)])
def test_host_basis_matches_oracle_interp(fcc, r, tau_max, D):
    p = fcc.Plan(np.array([[0, 0, 0], [0.15, 0, 0]]), 16000.0, frame_size=512, hop=256,
                 tau_max=tau_max, rank=D, interp=r)
    assert p.I == 2 * r * tau_max + 1
    e = p.basis_export()
    B = O.fcc_basis(512, tau_max, D, r)
    assert list(e["is_sym"]) == list(B.is_sym)
    assert np.abs(e["sigma"] - B.sigma).max() < 1e-12 * B.sigma[0]
    Ob = (B.Dc + 1j * B.Ds) @ (B.sigma[:, None] * B.v_full)
    assert np.abs(_operator(e, 512) - Ob).max() < 1e-12 * B.sigma[0]
    assert np.array_equal(e["Dc"], e["Dc"][::-1])
    assert np.array_equal(e["Ds"], -e["Ds"][::-1])


@pytest.mark.parametrize("xyz,fs,N,D", [
    (square_array(0.05), 16000.0, 512, 9),
    (circular_array(16, 0.05), 16000.0, 512, 6),
    (circular_array(16, 0.05), 16000.0, 512, 11),
    (circular_array(16, 0.05), 48000.0, 1024, 15),
    (circular_array(16, 0.05), 48000.0, 1024, 29),
    (circular_array(8, 0.04), 16000.0, 512, 5),
    (np.array([[0, 0, 0], [0.15, 0, 0]]), 16000.0, 512, 8),
])
def test_host_basis_matches_oracle(fcc, xyz, fs, N, D):
    p = fcc.Plan(xyz, fs, frame_size=N, hop=N // 4, rank=D)
    assert p.tau_max == O.tau_max_from_geometry(xyz, fs, 343.0)
    e = p.basis_export()
    B = O.fcc_basis(N, p.tau_max, D)
    assert list(e["is_sym"]) == list(B.is_sym)
    assert np.abs(e["sigma"] - B.sigma).max() < 1e-12 * B.sigma[0]
    # the rank-D subspace is unique (refused otherwise); vectors inside a
    # cluster of equal singular values are not, so compare the operator
    Ob = (B.Dc + 1j * B.Ds) @ (B.sigma[:, None] * B.v_full)
    assert np.abs(_operator(e, N) - Ob).max() < 1e-12 * B.sigma[0]
    # exact structure of the host tables
    m = N // 4
    for k in range(D):
        if not e["is_sym"][k]:
            assert e["p_hat"][k, m] == 0.0
    assert np.array_equal(e["Dc"], e["Dc"][::-1])
    assert np.array_equal(e["Ds"], -e["Ds"][::-1])


def test_mlp_host_queries(fcc):
    import oracle.mlp_oracle as MO
    from paper_2204_13622_amd.learned import learned_workspace_bytes
    lib = fcc._lib.load()
    for in_dim, H in [(10, 128), (22, 128), (64, 512), (1, 16)]:
        assert lib.fcc_mlp_num_params(in_dim, H) == MO.num_params(in_dim, H)
    b = ctypes.c_size_t()
    assert lib.fcc_mlp_workspace_bytes(10, 128, 1000, ctypes.byref(b)) == 0
    assert b.value == 4 * 1000 * (10 + 6 * 128 + 4)
    for bad in [(0, 128, 10), (65, 128, 10), (10, 40, 10), (10, 528, 10), (10, 128, -1)]:
        assert lib.fcc_mlp_workspace_bytes(*bad, ctypes.byref(b)) == -1, bad
    # argument errors return before any device work
    assert lib.fcc_mlp_forward(None, 10, 128, None, 5, None, None, None) == -1
    assert lib.fcc_mlp_adam(None, None, None, None, 5, 1e-3, 0.9, 0.999, 1e-8, 0, None) == -1
    p = fcc.Plan(circular_array(8, 0.04), 16000.0, frame_size=512, hop=512, rank=5)
    R = 100 * p.P
    # fused shape: coefficients and fallback lags only; other widths also hold the layers
    assert learned_workspace_bytes(p, 128, 100) >= 4 * R * (10 + 1)
    assert learned_workspace_bytes(p, 128, 100) < 4 * R * (10 + 6 * 128)
    assert learned_workspace_bytes(p, 48, 100) >= 4 * R * (10 + 1 + 2) + 4 * R * (10 + 6 * 48 + 4)
    assert learned_workspace_bytes(p, 128, 100) % 256 == 0
    with pytest.raises(fcc.FccError):
        learned_workspace_bytes(p, 100, 10)


def test_doa_table_matches_oracle(fcc):
    import oracle.doa_oracle as DO
    from gen import sphere_grid
    xyz = np.vstack([circular_array(6, 0.05), [[0.0, 0.0, 0.05]]])
    dirs = sphere_grid(300)
    for r in (1, 2):
        p = fcc.Plan(xyz, 16000.0, frame_size=512, hop=128, rank=5, interp=r)
        lib = fcc._lib.load()
        d = np.ascontiguousarray(dirs)
        tab = np.empty((p.P, d.shape[0]), dtype=np.float32)
        assert lib.fcc_doa_table(p._h, d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), d.shape[0],
                                 tab.ctypes.data_as(ctypes.c_void_p)) == 0
        q = DO.lag_positions(xyz, dirs, 16000.0, 343.0, p.tau_max, r)
        assert np.abs(tab - q).max() <= 4e-7 * p.I          # FP32 rounding of values below I
        bad = d.copy()
        bad[3, 1] = np.nan
        assert lib.fcc_doa_table(p._h, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), d.shape[0],
                                 tab.ctypes.data_as(ctypes.c_void_p)) == -1


def test_batch_validation_and_layout(fcc):
    from gen import batch_arrays
    arrays = batch_arrays(4000, 6, 0.3)
    plans = [fcc.Plan(a["xyz"], a["fs"], frame_size=a["N"], hop=a["hop"], rank=0, precision="fp16")
             for a in arrays]
    # the rank per geometry: tau_max + 1
    plans = [fcc.Plan(a["xyz"], a["fs"], frame_size=a["N"], hop=a["hop"], rank=p.tau_max + 1, precision="fp16")
             for a, p in zip(arrays, plans)]
    lengths = [a["x"].shape[1] for a in arrays]
    lib = fcc._lib.load()
    n = len(plans)
    h = ctypes.c_void_p()
    hs = (ctypes.c_void_p * n)(*[p._h for p in plans])
    ls = (ctypes.c_int64 * n)(*lengths)
    assert lib.fcc_batch_create(hs, n, ls, ctypes.byref(h)) == 0
    info = fcc._lib.FccBatchInfo()
    assert lib.fcc_batch_query(h, ctypes.byref(info)) == 0
    ao, to, nf = (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)()
    assert lib.fcc_batch_layout(h, ao, to, nf) == 0
    exp_a = np.cumsum([0] + [p.M * L for p, L in zip(plans, lengths)])
    exp_f = [p.num_frames(L) for p, L in zip(plans, lengths)]
    exp_t = np.cumsum([0] + [T * p.P for T, p in zip(exp_f, plans)])
    assert list(ao) == list(exp_a[:-1]) and info.audio_floats == exp_a[-1]
    assert list(nf) == exp_f and list(to) == list(exp_t[:-1]) and info.tdoa_count == exp_t[-1]
    assert info.num_arrays == n and 1 <= info.num_classes <= n
    assert info.image_bytes % 256 == 0 and info.workspace_bytes % 256 == 0
    lib.fcc_batch_destroy(h)
    # refusals
    bad = [plans[0], fcc.Plan(arrays[1]["xyz"], arrays[1]["fs"], frame_size=512, hop=128, precision="bf16")]
    hs = (ctypes.c_void_p * 2)(*[p._h for p in bad])
    assert lib.fcc_batch_create(hs, 2, (ctypes.c_int64 * 2)(100, 100), ctypes.byref(h)) == -1   # mixed precision
    for kw in [dict(precision="fp32"), dict(precision="fp16", alpha=0.5), dict(precision="fp16", method="gcc")]:
        q = fcc.Plan(square_array(0.05), 16000.0, **kw) if kw.get("alpha", 1.0) == 1.0 or kw.get("precision") == "fp32" \
            else None
        if q is None:
            continue
        hs = (ctypes.c_void_p * 1)(q._h)
        assert lib.fcc_batch_create(hs, 1, (ctypes.c_int64 * 1)(1000), ctypes.byref(h)) == -2, kw
    big = fcc.Plan(circular_array(17, 0.05), 16000.0, precision="fp16")
    hs = (ctypes.c_void_p * 1)(big._h)
    assert lib.fcc_batch_create(hs, 1, (ctypes.c_int64 * 1)(1000), ctypes.byref(h)) == -2
    # rank 32, three lag tiles at N = 1024: the tables and two slabs exceed 160 KB of LDS
    wide = fcc.Plan(circular_array(4, 0.05), 16000.0, frame_size=1024, hop=256, tau_max=20, rank=32, precision="fp16")
    hs = (ctypes.c_void_p * 1)(wide._h)
    assert lib.fcc_batch_create(hs, 1, (ctypes.c_int64 * 1)(4800), ctypes.byref(h)) == -2


def test_batch_classes_split_by_frame_size(fcc):
    """Pair-stage classes group arrays by tile shape and frame size: two
    arrays that differ only in N fall in two classes, equal ones in one."""
    lib = fcc._lib.load()
    xyz = square_array(0.05)
    mk = lambda N: fcc.Plan(xyz, 16000.0, frame_size=N, hop=N // 4, rank=4, precision="fp16")  # noqa: E731
    for sizes, classes in [((512, 512), 1), ((256, 512), 2), ((256, 512, 1024, 512), 3)]:
        plans = [mk(N) for N in sizes]
        n = len(plans)
        h = ctypes.c_void_p()
        hs = (ctypes.c_void_p * n)(*[p._h for p in plans])
        assert lib.fcc_batch_create(hs, n, (ctypes.c_int64 * n)(*([4000] * n)), ctypes.byref(h)) == 0
        info = fcc._lib.FccBatchInfo()
        assert lib.fcc_batch_query(h, ctypes.byref(info)) == 0
        assert info.num_classes == classes, sizes
        lib.fcc_batch_destroy(h)


def test_batch_layout_with_arrays_without_frames(fcc):
    """Arrays shorter than their frame size get no frames and no output span;
    a negative length is refused."""
    lib = fcc._lib.load()
    xyz = square_array(0.05)
    plans = [fcc.Plan(xyz, 16000.0, frame_size=N, hop=N // 4, rank=4, precision="fp16") for N in (512, 256, 512)]
    n = len(plans)
    hs = (ctypes.c_void_p * n)(*[p._h for p in plans])
    for lengths, frames in [((511, 256, 0), (0, 1, 0)), ((0, 0, 0), (0, 0, 0)), ((512, 100, 640), (1, 0, 2))]:
        h = ctypes.c_void_p()
        assert lib.fcc_batch_create(hs, n, (ctypes.c_int64 * n)(*lengths), ctypes.byref(h)) == 0
        info = fcc._lib.FccBatchInfo()
        assert lib.fcc_batch_query(h, ctypes.byref(info)) == 0
        ao, to, nf = (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)()
        assert lib.fcc_batch_layout(h, ao, to, nf) == 0
        assert tuple(nf) == frames
        assert list(to) == list(np.cumsum([0] + [T * p.P for T, p in zip(frames, plans)])[:-1])
        assert info.tdoa_count == sum(T * p.P for T, p in zip(frames, plans))
        assert info.audio_floats == sum(p.M * L for p, L in zip(plans, lengths))
        lib.fcc_batch_destroy(h)
    h = ctypes.c_void_p()
    assert lib.fcc_batch_create(hs, n, (ctypes.c_int64 * n)(512, -1, 512), ctypes.byref(h)) == -1
