"""Host-side checks of the C-ABI library: symbols, validation, plan tables.

Nothing here launches a kernel; plan creation and its accessors run on the
CPU only.
"""
import ctypes

import numpy as np
import pytest

import oracle as O
import paper_2501_04684_amd as U
import workloads as W

A, K = 0.25, 2 * np.pi


def test_library_exports_every_declared_symbol():
    L = U.lib()
    names = U.declared_symbols()
    assert len(names) == 34
    for name in names:
        assert hasattr(L, name), name


def test_status_strings():
    assert U.status_string(0) == "ok"
    for st in (-1, -2, -3, -4):
        assert U.status_string(st) not in ("ok", "unknown status")
    assert U.status_string(-99) == "unknown status"


@pytest.mark.parametrize("kwargs,msg", [
    (dict(boxes=np.zeros((0, 3))), "n_boxes"),
    (dict(boxes=np.array([[0, 0, 0], [0, 0, 0]])), "duplicate"),
    (dict(boxes=np.array([[0, -1, 0]])), ">= 0"),
    (dict(a=0.0), "box side"),
    (dict(a=-1.0), "box side"),
    (dict(k=0.0), "wavenumber"),
    (dict(k=float("nan")), "wavenumber"),
    (dict(n_d=0), "n_d"),
    (dict(n_d=5), "n_d"),
    (dict(far_mode=7), "far_mode"),
    (dict(eta=-1.0), "eta"),
])
def test_plan_create_rejects(kwargs, msg):
    args = dict(boxes=W.grid_boxes(2, 2, 2), a=A, k=K, n_d=3, far_mode="ilist")
    args.update(kwargs)
    fm = args.pop("far_mode")
    boxes = args.pop("boxes")
    if isinstance(fm, int) and fm not in (0, 1):
        b = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32))
        prob = U._Problem(len(b), b.ctypes.data, args["a"], args["k"], 0.0,
                          args["n_d"], fm, 0)
        out = ctypes.c_void_p()
        st = U.lib().ubf_plan_create(ctypes.byref(prob), ctypes.byref(out))
        assert st == -1 and msg in U.last_error() and not out.value
        return
    with pytest.raises(U.UbfError) as e:
        U.plan_create(boxes, far_mode=fm, **args)
    assert e.value.status == -1
    assert msg in str(e.value)


def test_null_arguments_rejected_before_any_device_call():
    L = U.lib()
    out = ctypes.c_void_p()
    assert L.ubf_plan_create(None, ctypes.byref(out)) == -1
    assert L.ubf_workspace_bytes(None, 1) == 0
    assert L.ubf_plan_bind(None, None, 0, 1, None) == -1
    assert L.ubf_far_mvm(None, None, None, 1, None) == -1
    assert L.ubf_plan_info(None, None) == -1
    assert L.ubf_profile_begin(None, 1, 1) == -1
    assert L.ubf_profile_end(None, None, None, None) == -1
    plan = U.plan_create(W.grid_boxes(2, 2, 2), A, K, 2)
    try:
        # unbound plan: state error, not a device call
        assert L.ubf_far_mvm(plan, 1 << 20, 2 << 20, 1, None) == -4
        assert L.ubf_translate(plan, 1 << 20, 2 << 20, 1, None) == -4
        assert L.ubf_plan_set_basis(plan, None, None, None) == -4
        # bad workspace: misaligned, too small
        assert L.ubf_plan_bind(plan, 1 << 20 | 8, 1 << 30, 1, None) == -1
        assert L.ubf_plan_bind(plan, 1 << 20, 16, 1, None) == -2
        assert "too small" in U.last_error()
        assert L.ubf_plan_bind(plan, 1 << 20, 1 << 30, 0, None) == -1
        assert L.ubf_workspace_bytes(plan, 0) == 0
        assert L.ubf_plan_operator(plan, 10 ** 6, None) == -1
        assert L.ubf_profile_begin(plan, 0, 1) == -1
        assert L.ubf_profile_begin(plan, 1, 0) == -1
        assert L.ubf_profile_end(plan, None, None, None) == -4
        # networks: unbound plan is a state error; hidden 0 always clears
        assert L.ubf_plan_set_networks(plan, 16, 1 << 20, 1 << 20, 1 << 20, 1 << 20,
                                       1 << 20, 1 << 30, None) == -4
        assert L.ubf_plan_set_networks(plan, 0, None, None, None, None, None, 0, None) == 0
    finally:
        U.plan_destroy(plan)
    assert L.ubf_network_bytes(None, 16) == 0
    assert L.ubf_plan_set_networks(None, 16, None, None, None, None, None, 0, None) == -1


@pytest.mark.parametrize("n_d,ok", [(1, False), (2, True), (3, True), (4, True)])
def test_network_image_size(n_d, ok):
    plan = U.plan_create(W.grid_boxes(4, 4, 2), A, K, n_d)
    try:
        n_off = U.plan_info(plan)["n_offsets"]
        for hidden in (1, 32, 33, 50, 64):
            nb = U.network_bytes(plan, hidden)
            assert (nb > 0) == ok
            if ok:
                assert nb % (16 * n_off) == 0
        # wider networks never take less room; out-of-range widths have no kernel
        if ok:
            assert U.network_bytes(plan, 33) > U.network_bytes(plan, 32)
        assert U.network_bytes(plan, 0) == 0
        assert U.network_bytes(plan, 65) == 0
    finally:
        U.plan_destroy(plan)


@pytest.mark.parametrize("cfg", [1, 2])
def test_plan_far_set_matches_oracle(cfg):
    w = W.config(cfg)
    plan = U.plan_create(w.boxes, w.a, w.k, w.n_d, w.far_mode)
    try:
        info = U.plan_info(plan)
        j, i, off = O.far_pairs(w.boxes, w.far_mode)
        uniq, _ = O.offset_ids(off)
        assert info["n_pairs"] == len(j)
        assert info["n_offsets"] == len(uniq)
        assert info["n_orbits"] == len(O.symmetry.orbits(uniq))
        assert info["n_u"] == 81 and info["mfma"] == 1
        assert info["translate_flops"] == 8 * 81 * 81 * len(j)
        t, s, o = U.plan_far_pairs(plan)
        offs = U.plan_offsets(plan)
        got = sorted(zip(t.tolist(), s.tolist(), map(tuple, offs[o].tolist())))
        ref = sorted(zip(j.tolist(), i.tolist(), map(tuple, off.tolist())))
        assert got == ref
        # grouped by offset, each offset's pairs in test-box order
        assert np.all(np.diff(o) >= 0)
        for oo in np.unique(o)[:20]:
            assert np.all(np.diff(t[o == oo]) > 0)
        # the work partition covers every pair once
        assert info["n_chunks"] >= -(-len(j) // 128)
        # items of the LDS-staged kernels: each offset's pairs in pieces of 32
        _, per_off = np.unique(off, axis=0, return_counts=True)
        assert info["n_items"] == int(np.sum(-(-per_off // 32)))
        assert info["n_chunks"] == int(np.sum(-(-per_off // 128)))
    finally:
        U.plan_destroy(plan)


def test_full_mode_and_orbits():
    b = W.grid_boxes(6, 6, 6)
    plan = U.plan_create(b, A, K, 1, "full")
    try:
        info = U.plan_info(plan)
        assert (info["n_pairs"], info["n_offsets"], info["n_orbits"]) == (42560, 1304, 52)
    finally:
        U.plan_destroy(plan)


@pytest.mark.parametrize("n_d", [1, 2, 3, 4])
def test_host_operators_match_oracle(n_d):
    b = W.grid_boxes(4, 4, 4)
    plan = U.plan_create(b, A, K, n_d, "ilist")
    try:
        offs = U.plan_offsets(plan)
        for o in (0, 7, 100, 315):
            G = U.plan_operator(plan, o)
            ref = O.translation_operator(offs[o], A, K, n_d)
            assert np.abs(G - ref).max() <= 1e-13 * np.abs(ref).max()
    finally:
        U.plan_destroy(plan)


def test_low_frequency_operator():
    # a = lambda/256 regime of the low-frequency example (Sec. 5)
    b = W.grid_boxes(4, 4, 4)
    a = 1.0 / 256
    plan = U.plan_create(b, a, K, 3, "ilist", eta=1.0)
    try:
        offs = U.plan_offsets(plan)
        for o in (0, 200):
            G = U.plan_operator(plan, o)
            ref = O.translation_operator(offs[o], a, K, 3, eta=1.0)
            assert np.abs(G - ref).max() <= 1e-12 * np.abs(ref).max()
    finally:
        U.plan_destroy(plan)


def test_workspace_grows_with_nrhs():
    plan = U.plan_create(W.grid_boxes(4, 4, 4), A, K, 3)
    try:
        w1, w2 = U.workspace_bytes(plan, 1), U.workspace_bytes(plan, 2)
        assert 0 < w1 < w2 and w1 % 256 == 0
    finally:
        U.plan_destroy(plan)


def test_sparse_coordinates_use_hash_index():
    # coordinates far apart: dense index grid would be enormous
    b = np.array([[0, 0, 0], [0, 0, 2], [4000, 4000, 4000], [4000, 4000, 4003]])
    plan = U.plan_create(b, A, K, 1, "full")
    try:
        t, s, _ = U.plan_far_pairs(plan)
        j, i, _ = O.far_pairs(b, "full")
        assert sorted(zip(t, s)) == sorted(zip(j, i))
    finally:
        U.plan_destroy(plan)


def _lib_pairs(b, mode):
    plan = U.plan_create(b, A, K, 1, mode)
    try:
        t, s, o = U.plan_far_pairs(plan)
        offs = U.plan_offsets(plan)
        return sorted(zip(t.tolist(), s.tolist(), map(tuple, offs[o].tolist())))
    finally:
        U.plan_destroy(plan)


def _oracle_pairs(b, mode):
    j, i, w = O.far_pairs(b, mode)
    return sorted(zip(j.tolist(), i.tolist(), map(tuple, w.tolist())))


@pytest.mark.parametrize("boxes", [
    # z = 2^21 + 2 once shared a packed hash key with (0, 1, 2): a spurious
    # ILIST pair two million boxes apart
    [[0, 1, 0], [0, 0, 2**21 + 2], [7, 0, 0]],
    # z = 2^21 once collided with (0, 1, 0): a false duplicate
    [[0, 0, 2**21], [0, 1, 0], [5, 0, 0]],
])
@pytest.mark.parametrize("mode", ["ilist", "full"])
def test_far_set_exact_at_large_coordinates(boxes, mode):
    # Algorithm 2 on boxes whose coordinates exceed 21 bits: the sparse box
    # index must compare whole coordinates (Sec. 2 box partition)
    b = np.array(boxes, dtype=np.int32)
    assert _lib_pairs(b, mode) == _oracle_pairs(b, mode)


def _clusters(rng, n_clusters):
    """Random occupancy of small blocks placed at large, colliding coordinates."""
    base_choices = [0, 2**21, 2**21 - 2, 2**22, 2**30, 2**31 - 8, 4000]
    parts, origins = [], []
    for _ in range(n_clusters):
        while True:
            org = np.array([rng.choice(base_choices) for _ in range(3)], dtype=np.int64)
            org -= org % 2  # even origins keep the ILIST parent rule intact
            org = np.minimum(org, 2**31 - 8)
            if all(np.abs(org - o).max() > 8 for o in origins):
                break
        origins.append(org)
        ext = rng.integers(2, 6, size=3)
        g = np.stack(np.meshgrid(*[np.arange(e) for e in ext], indexing="ij"),
                     axis=-1).reshape(-1, 3)
        g = g[rng.random(len(g)) < rng.uniform(0.3, 1.0)]
        if len(g) == 0:
            g = np.zeros((1, 3), dtype=np.int64)
        parts.append((org, g))
    return parts


@pytest.mark.parametrize("seed", range(6))
def test_far_set_random_sparse_geometries(seed):
    # Seeded clusters at coordinates up to 2^31 - 1 (sparse index path):
    # ILIST never joins clusters more than three boxes apart, so the oracle
    # runs per cluster on even-shifted coordinates, which leaves the parent
    # rule floor(c/2) unchanged; FULL runs the oracle on the whole set.
    rng = np.random.default_rng(1000 + seed)
    parts = _clusters(rng, int(rng.integers(2, 5)))
    b = np.concatenate([org + g for org, g in parts]).astype(np.int64)
    perm = rng.permutation(len(b))
    b = b[perm]
    inv = np.argsort(perm)
    assert b.max() <= 2**31 - 1
    ref, start = [], 0
    for org, g in parts:
        j, i, w = O.far_pairs(g, "ilist")
        ref += [(int(inv[start + jj]), int(inv[start + ii]), tuple(ww))
                for jj, ii, ww in zip(j.tolist(), i.tolist(), w.tolist())]
        start += len(g)
    assert _lib_pairs(b.astype(np.int32), "ilist") == sorted(ref)
    assert _lib_pairs(b.astype(np.int32), "full") == _oracle_pairs(b, "full")


def test_split_precision_plan():
    b = W.grid_boxes(4, 4, 4)
    plan = U.plan_create(b, A, K, 3, "ilist", precision="split-bf16")
    try:
        info = U.plan_info(plan)
        assert info["precision"] == U.SPLIT_BF16
        # four BF16 planes of 81 x 88 per offset
        assert info["table_bytes"] == info["n_offsets"] * 4 * 81 * 88 * 2
    finally:
        U.plan_destroy(plan)
    # 192 coefficients per box (the paper's 4x4x4 dipoles): the operator in
    # the staged kernel's fragment order, 12 row blocks x 24 k-steps x (hi,
    # lo) x 64 lanes x 8 values; the single FP16 product keeps hi only
    for form, parts in (("split-bf16", 2), ("split-fp16", 2), ("fp16", 1)):
        plan = U.plan_create(b, 0.125, K, 4, "ilist", precision=form)
        try:
            info = U.plan_info(plan)
            assert info["n_u"] == 192 and info["mfma"] == 1
            assert info["table_bytes"] == info["n_offsets"] * 12 * 24 * parts * 64 * 8 * 2
        finally:
            U.plan_destroy(plan)


def test_generated_operator_plans():
    # operators evaluated by the stage-2 kernel: no table in the plan or the
    # workspace (the workspace shrinks by the table's bytes, up to their
    # 256-byte alignment), the same far set; only the 16-bit forms with n_d
    # 1..3 accept it
    b = W.grid_boxes(6, 6, 6)
    for form in ("split-bf16", "split-fp16", "fp16"):
        tab = U.plan_create(b, A, K, 3, "full", precision=form)
        gen = U.plan_create(b, A, K, 3, "full", precision=form, operators="generated")
        try:
            ti, gi = U.plan_info(tab), U.plan_info(gen)
            assert ti["operators"] == U.OPERATORS_TABLE and gi["operators"] == U.OPERATORS_GENERATED
            assert gi["table_bytes"] == 0 and ti["table_bytes"] > 0
            assert (gi["n_pairs"], gi["n_offsets"], gi["n_chunks"]) == \
                (ti["n_pairs"], ti["n_offsets"], ti["n_chunks"])
            assert np.array_equal(U.plan_offsets(gen), U.plan_offsets(tab))
            saved = U.workspace_bytes(tab, 1) - U.workspace_bytes(gen, 1)
            assert 0 <= saved - ti["table_bytes"] < 256
            # host introspection still evaluates operators on demand
            G = U.plan_operator(gen, 0)
            assert np.allclose(G, U.plan_operator(tab, 0), rtol=0, atol=0)
        finally:
            U.plan_destroy(tab)
            U.plan_destroy(gen)
    for kw in (dict(precision="fp32"), dict(n_d=4, precision="split-fp16")):
        args = dict(n_d=3)
        args.update(kw)
        with pytest.raises(U.UbfError) as e:
            U.plan_create(b, 0.125, K, args.pop("n_d"), "ilist", operators="generated", **args)
        assert e.value.status == -1 and "generated operators" in str(e.value)
    bi = np.ascontiguousarray(b.astype(np.int32))
    prob = U._Problem(len(bi), bi.ctypes.data, A, K, 0.0, 3, 0, 2, 7)
    out = ctypes.c_void_p()
    assert U.lib().ubf_plan_create(ctypes.byref(prob), ctypes.byref(out)) == -1
    assert "operator source" in U.last_error() and not out.value


def _small_scatterers():
    return [b for _, b in W.scatterer_set(6, seed=11, lo=40, hi=300)]


def test_batch_far_set_is_union_of_solo_far_sets():
    parts = _small_scatterers()
    plan = U.plan_create_batch(parts, A, K, 3)
    try:
        info = U.plan_info(plan)
        assert info["n_scatterers"] == len(parts)
        assert info["n_boxes"] == sum(len(b) for b in parts)
        t, s, o = U.plan_far_pairs(plan)
        offs = U.plan_offsets(plan)
        got = set(zip(t.tolist(), s.tolist(), map(tuple, offs[o].tolist())))
        want = set()
        base = 0
        union_offsets = set()
        for b in parts:
            # the oracle's far set of this scatterer alone, shifted to the
            # batch numbering
            j, i, w = O.far_pairs(b, O.FAR_ILIST)
            want |= set(zip((j + base).tolist(), (i + base).tolist(), map(tuple, w.tolist())))
            union_offsets |= set(map(tuple, w.tolist()))
            base += len(b)
        assert got == want
        assert set(map(tuple, offs.tolist())) == union_offsets
        # no pair joins two scatterers
        ptr = np.cumsum([0] + [len(b) for b in parts])
        assert (np.searchsorted(ptr, t, "right") == np.searchsorted(ptr, s, "right")).all()
    finally:
        U.plan_destroy(plan)


def test_batch_matches_solo_plans_pair_for_pair():
    parts = _small_scatterers()
    plan = U.plan_create_batch(parts, A, K, 3, far_mode="full")
    base = 0
    try:
        t, s, o = U.plan_far_pairs(plan)
        offs = U.plan_offsets(plan)
        for b in parts:
            solo = U.plan_create(b, A, K, 3, far_mode="full")
            try:
                ts, ss, os_ = U.plan_far_pairs(solo)
                sel = (t >= base) & (t < base + len(b))
                got = sorted(zip((t[sel] - base).tolist(), (s[sel] - base).tolist(),
                                 map(tuple, offs[o[sel]].tolist())))
                so = U.plan_offsets(solo)
                want = sorted(zip(ts.tolist(), ss.tolist(), map(tuple, so[os_].tolist())))
                assert got == want
            finally:
                U.plan_destroy(solo)
            base += len(b)
    finally:
        U.plan_destroy(plan)


def test_batch_repeated_coordinates_across_scatterers():
    g = W.grid_boxes(4, 4, 4)
    plan = U.plan_create_batch([g, g, g], A, K, 2)
    try:
        info = U.plan_info(plan)
        solo = U.plan_create(g, A, K, 2)
        assert info["n_pairs"] == 3 * U.plan_info(solo)["n_pairs"]
        U.plan_destroy(solo)
    finally:
        U.plan_destroy(plan)


@pytest.mark.parametrize("ptr,msg", [
    ([0, 0, 8], "at least one box"),
    ([0, 4, 7], "must equal n_boxes"),
    ([1, 4, 8], "scatterer_ptr[0]"),
    ([0, 5, 4, 8], "at least one box"),
])
def test_batch_rejects_bad_scatterer_ptr(ptr, msg):
    b = np.ascontiguousarray(W.grid_boxes(2, 2, 2))
    prob = U._Problem(len(b), b.ctypes.data, A, K, 0.0, 3, 0, 0)
    p = np.asarray(ptr, dtype=np.int64)
    out = ctypes.c_void_p()
    st = U.lib().ubf_plan_create_batch(ctypes.byref(prob), len(p) - 1, p.ctypes.data,
                                       ctypes.byref(out))
    assert st == -1 and msg in U.last_error() and not out.value
    st = U.lib().ubf_plan_create_batch(ctypes.byref(prob), 2, None, ctypes.byref(out))
    assert st == -1 and "scatterer_ptr" in U.last_error()


def test_batch_duplicate_within_one_scatterer_rejected():
    g = W.grid_boxes(2, 2, 2)
    with pytest.raises(U.UbfError, match="duplicate"):
        U.plan_create_batch([g, np.concatenate([g, g[:1]])], A, K, 3)


def test_graph_and_tune_need_a_bound_plan():
    plan = U.plan_create(W.grid_boxes(4, 4, 4), A, K, 3)
    try:
        L = U.lib()
        assert L.ubf_plan_replay(plan, None) == -4
        assert "no captured" in U.last_error()
        assert L.ubf_plan_tune(plan, 1, 3, None, None) == -4
        assert L.ubf_plan_capture(plan, 16, 1 << 20, 1) == -4
        assert L.ubf_plan_replay(None, None) == -1
        info = U.plan_info(plan)
        assert info["translate_groups"] % 8 == 0 and info["n_scatterers"] == 1
    finally:
        U.plan_destroy(plan)


def test_gmres_checks_before_any_device_call():
    plan = U.plan_create(W.grid_boxes(3, 3, 3), A, K, 2)
    try:
        L = U.lib()
        out = ctypes.c_void_p()
        fake = 1 << 20  # aligned, never dereferenced: the plan is unbound
        assert U.gmres_workspace_bytes(plan, 1, 100) > 0
        assert U.gmres_workspace_bytes(plan, 1, 129) == 0
        assert U.gmres_workspace_bytes(plan, 0, 10) == 0
        st = L.ubf_gmres_create(plan, 1, 10, 1.0, 0.0, 1e-4, 10, fake, 1 << 30,
                                ctypes.byref(out))
        assert st == -4 and "not bound" in U.last_error() and not out.value
        for args, msg in [((0, 10), "nrhs"), ((1, 0), "restart"), ((1, 200), "restart")]:
            st = L.ubf_gmres_create(plan, args[0], args[1], 1.0, 0.0, 1e-4, 10, fake,
                                    1 << 30, ctypes.byref(out))
            assert st == -1 and msg in U.last_error()
        st = L.ubf_gmres_create(plan, 1, 10, 1.0, 0.0, 0.0, 10, fake, 1 << 30,
                                ctypes.byref(out))
        assert st == -1 and "tol" in U.last_error()
        st = L.ubf_gmres_create(plan, 1, 10, 1.0, 0.0, 1e-4, 10, fake + 4, 1 << 30,
                                ctypes.byref(out))
        assert st == -1 and "aligned" in U.last_error()
        assert L.ubf_gmres_step(None, None) == -1
    finally:
        U.plan_destroy(plan)


@pytest.mark.parametrize("form,code", [("split-fp16", 2), ("fp16", 3)])
def test_fp16_plans(form, code):
    b = W.grid_boxes(4, 4, 4)
    plan = U.plan_create(b, A, K, 3, "ilist", precision=form)
    try:
        info = U.plan_info(plan)
        assert info["precision"] == code
        assert info["table_bytes"] == info["n_offsets"] * 4 * 81 * 88 * 2
    finally:
        U.plan_destroy(plan)
    # n_d = 4 is accepted in every form (see test_split_precision_plan);
    # an unknown precision code is refused
    bb = np.ascontiguousarray(b.astype(np.int32))
    prob = U._Problem(len(bb), bb.ctypes.data, A, K, 0.0, 3, 0, 4)
    out = ctypes.c_void_p()
    assert U.lib().ubf_plan_create(ctypes.byref(prob), ctypes.byref(out)) == -1
    assert "precision" in U.last_error()
