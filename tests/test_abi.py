"""CPU-only checks of the C ABI: the library loads, exports every function
include/gbmc.h declares, and its host-side validation and scheduling behave.
No compute call is made (there is no GPU here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gbmc.h")


@pytest.fixture(scope="module")
def L():
    from paper_1803_09652_amd import _lib
    _lib.load()
    return _lib


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:gbmc_status|void|size_t|int32_t|const char\*)\s+(\w+)\s*\(",
                       text, flags=re.M)
    return names


def test_every_declared_symbol_is_exported_and_bound(L):
    names = header_functions()
    assert len(names) >= 18
    lib = C.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(L.SIGNATURES), "binding and header disagree"


def test_missing_library_fails_loudly(monkeypatch, L):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", "/nonexistent/libgbmc.so")
    with pytest.raises(RuntimeError, match="not built"):
        L.load()


def _i32p(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def test_params_validation(L):
    lib = L.load()
    ok = L.gbmc_gb_params(1.0, 0.8, 4.85, 0.09, 1.0, 78.5, 332.0522, 0.0, 0.0, 0.0)
    assert lib.gbmc_params_validate(C.byref(ok)) == L.GBMC_OK
    salt = L.gbmc_gb_params(1.0, 0.8, 4.85, 0.09, 1.0, 78.5, 332.0522, 0.1, 12.0, 15.0)
    assert lib.gbmc_params_validate(C.byref(salt)) == L.GBMC_OK
    neg = L.gbmc_gb_params(1.0, 0.8, 4.85, 0.09, 1.0, 78.5, 332.0522, -0.1, 0.0, 0.0)
    assert lib.gbmc_params_validate(C.byref(neg)) == L.GBMC_ERR_INVALID
    assert b"kappa" in lib.gbmc_last_error()
    negc = L.gbmc_gb_params(1.0, 0.8, 4.85, 0.09, 1.0, 78.5, 332.0522, 0.0, -1.0, 0.0)
    assert lib.gbmc_params_validate(C.byref(negc)) == L.GBMC_ERR_INVALID
    bad = L.gbmc_gb_params(1.0, 0.8, 4.85, 0.09, 0.0, 78.5, 332.0522, 0.0, 0.0, 0.0)
    assert lib.gbmc_params_validate(C.byref(bad)) == L.GBMC_ERR_INVALID
    nan = L.gbmc_gb_params(float("nan"), 0.8, 4.85, 0.09, 1.0, 78.5, 332.0522, 0.0, 0.0, 0.0)
    assert lib.gbmc_params_validate(C.byref(nan)) == L.GBMC_ERR_INVALID


def schedule(L, off, jb=None, row_pairs=1):
    lib = L.load()
    off = np.ascontiguousarray(off, dtype=np.int32)
    n = C.c_int32()
    jb = jb or 8
    st = lib.gbmc_schedule_build(off.size - 1, _i32p(off), jb, row_pairs, C.byref(n), None)
    if st != 0:
        return st, None
    items = np.zeros(5 * n.value, dtype=np.int32)
    assert lib.gbmc_schedule_build(off.size - 1, _i32p(off), jb, row_pairs, C.byref(n),
                                   _i32p(items)) == 0
    return st, items.reshape(-1, 5)


@pytest.mark.parametrize("row_pairs", [1, 0])
@pytest.mark.parametrize("jb", [None, 1, 3, 8, 1000])
def test_schedule_covers_every_tile_once(L, jb, row_pairs):
    sizes = [1, 64, 65, 0, 200, 2500, 130, 129]
    off = np.concatenate([[0], np.cumsum(sizes)])
    st, items = schedule(L, off, jb, row_pairs)
    assert st == 0
    seen = {}
    for sys_, I0, I1, J0, J1 in items:
        rows = I1 - I0
        assert rows in ((1, 2) if row_pairs else (1,))
        assert 0 <= I0 <= J0 < J1
        if rows == 2:
            assert I0 % 2 == 0 and J0 >= I0 + 2
        if jb:
            assert J1 - J0 <= jb
        for I in range(I0, I1):
            for J in range(J0, J1):
                key = (sys_, I, J)
                assert key not in seen
                seen[key] = 1
    for b, n in enumerate(sizes):
        nb = (n + 63) // 64
        for I in range(nb):
            for J in range(I, nb):
                assert (b, I, J) in seen
    assert len(seen) == sum(((n + 63) // 64) * ((n + 63) // 64 + 1) // 2 for n in sizes)
    # longest first, in half tiles
    rows = items[:, 2] - items[:, 1]
    cost = 2 * rows * (items[:, 4] - items[:, 3]) - (items[:, 3] == items[:, 1])
    assert np.all(np.diff(cost) <= 0)


def test_schedule_rejects_bad_offsets(L):
    lib = L.load()
    n = C.c_int32()
    off = np.array([0, 10], dtype=np.int32)
    assert lib.gbmc_schedule_build(1, _i32p(off), 0, 1, C.byref(n), None) == L.GBMC_ERR_INVALID
    assert schedule(L, [1, 5])[0] == L.GBMC_ERR_INVALID
    assert schedule(L, [0, 5, 3])[0] == L.GBMC_ERR_INVALID
    st, items = schedule(L, [0])
    assert st == 0 and items.size == 0


def test_plan_create_rejects_bad_layout_before_touching_the_gpu(L):
    lib = L.load()
    h = C.c_void_p()
    off = np.array([0, 10, 5], dtype=np.int32)
    assert lib.gbmc_plan_create(C.byref(h), 2, _i32p(off), 0, None) == L.GBMC_ERR_INVALID
    off = np.array([0, 10], dtype=np.int32)
    assert lib.gbmc_plan_create(C.byref(h), 1, _i32p(off), 7, None) == L.GBMC_ERR_INVALID
    from paper_1803_09652_amd.api import tuning_struct
    bad = C.byref(tuning_struct((1, 0, 1), 4))
    assert lib.gbmc_plan_create(C.byref(h), 1, _i32p(off), 0, bad) == L.GBMC_ERR_INVALID
    bad = C.byref(tuning_struct(8, (1, 3, 1)))
    assert lib.gbmc_plan_create(C.byref(h), 1, _i32p(off), 0, bad) == L.GBMC_ERR_INVALID


def _sites_args(batch):
    return (batch.n_systems, _i32p(batch.atom_offset), batch.n_sites, _i32p(batch.site_system),
            _i32p(batch.site_kind), _i32p(batch.site_atom_offset), _i32p(batch.site_atoms),
            _i32p(batch.site_state_offset), _i32p(batch.state_charge_offset),
            _i32p(batch.state_count))


def test_sites_validation(L):
    lib = L.load()
    batch = synth.make_batch(synth.eremd_batch(n_rep=3))
    assert lib.gbmc_sites_validate(*_sites_args(batch)) == L.GBMC_OK
    # overlapping sites
    b2 = synth.make_batch(synth.eremd_batch(n_rep=3))
    b2.site_atoms[b2.site_atom_offset[1]] = b2.site_atoms[0]
    assert lib.gbmc_sites_validate(*_sites_args(b2)) == L.GBMC_ERR_INVALID
    assert b"overlap" in lib.gbmc_last_error()
    # atom outside its system
    b3 = synth.make_batch(synth.eremd_batch(n_rep=3))
    b3.site_atoms[0] = b3.atom_offset[2] + 1
    assert lib.gbmc_sites_validate(*_sites_args(b3)) == L.GBMC_ERR_INVALID
    # a one-state site
    s = synth.make_system(1, 100, 8.0, n_redox=1, redox_atoms=5)
    s.sites[0].charges = s.sites[0].charges[:1]
    s.sites[0].counts = s.sites[0].counts[:1]
    b4 = synth.make_batch([s])
    assert lib.gbmc_sites_validate(*_sites_args(b4)) == L.GBMC_ERR_UNSUPPORTED
    # more than 256 atoms in a site
    big = synth.make_system(2, 400, 12.0, n_redox=1, redox_atoms=300)
    assert lib.gbmc_sites_validate(*_sites_args(synth.make_batch([big]))) == L.GBMC_ERR_UNSUPPORTED
    # systems out of order
    b5 = synth.make_batch(synth.eremd_batch(n_rep=3))
    b5.site_system[0] = 2
    assert lib.gbmc_sites_validate(*_sites_args(b5)) == L.GBMC_ERR_INVALID


def test_exchange_rejects_bad_arguments_on_host(L):
    lib = L.load()
    assert lib.remd_exchange(4, None, None, None, 300.0, 2, 1, None, None, None, None) == L.GBMC_ERR_INVALID
    assert lib.remd_exchange(4, None, None, None, -1.0, 0, 1, None, None, None, None) == L.GBMC_ERR_INVALID
    assert lib.remd_exchange(4, None, None, None, 300.0, 0, 1, None, None, None, None) == L.GBMC_ERR_INVALID
    # one replica: nothing to do, no device access
    assert lib.remd_exchange(1, None, None, None, 300.0, 0, 1, None, None, None, None) == L.GBMC_OK


def test_entry_points_reject_null_plan(L):
    lib = L.load()
    p = L.gbmc_gb_params(1.0, 0.8, 4.85, 0.09, 1.0, 78.5, 332.0522, 0.0, 0.0, 0.0)
    a = L.gbmc_atoms()
    assert lib.gb_radii(None, C.byref(a), C.byref(p), None, None, None) == L.GBMC_ERR_INVALID
    assert lib.gb_energy_forces(None, C.byref(a), C.byref(p), None, None, None, None, None, None,
                                None) == L.GBMC_ERR_INVALID


def test_spatial_order_is_a_local_permutation(L):
    lib = L.load()
    systems = synth.eremd_batch(n_rep=3)
    batch = synth.make_batch(systems)
    off = batch.atom_offset
    out = np.zeros(batch.n_atoms, dtype=np.int32)
    d = lambda a: np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(C.POINTER(C.c_double))
    assert lib.gbmc_spatial_order(batch.n_systems, _i32p(off), d(batch.x), d(batch.y), d(batch.z),
                                  _i32p(out)) == 0
    xyz = np.stack([batch.x, batch.y, batch.z], 1)
    for b in range(batch.n_systems):
        seg = out[off[b]:off[b + 1]]
        assert sorted(seg.tolist()) == list(range(off[b], off[b + 1]))
        # consecutive atoms in the order are much closer than in the input order
        step = np.linalg.norm(np.diff(xyz[seg], axis=0), axis=1).mean()
        step0 = np.linalg.norm(np.diff(xyz[off[b]:off[b + 1]], axis=0), axis=1).mean()
        assert step < 0.4 * step0


def test_block_order_gives_compact_blocks(L):
    lib = L.load()
    systems = [synth.make_system(150, 3000, 20.0), synth.make_system(151, 130, 6.0),
               synth.make_system(152, 1, 2.0), synth.make_system(153, 64, 5.0)]
    batch = synth.make_batch(systems)
    off = batch.atom_offset
    out = np.zeros(batch.n_atoms, dtype=np.int32)
    d = lambda a: np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(C.POINTER(C.c_double))
    assert lib.gbmc_block_order(batch.n_systems, _i32p(off), d(batch.x), d(batch.y), d(batch.z),
                                _i32p(out)) == 0
    xyz = np.stack([batch.x, batch.y, batch.z], 1)

    def radii_of(seg):
        r = []
        for k in range(0, seg.size, 64):
            blk = xyz[seg[k:k + 64]]
            c = 0.5 * (blk.min(0) + blk.max(0))
            r.append(np.sqrt(((blk - c) ** 2).sum(1)).max())
        return np.array(r)

    for b in range(batch.n_systems):
        seg = out[off[b]:off[b + 1]]
        assert sorted(seg.tolist()) == list(range(off[b], off[b + 1]))
    seg = out[off[0]:off[1]]
    morton = np.zeros(batch.n_atoms, dtype=np.int32)
    assert lib.gbmc_spatial_order(batch.n_systems, _i32p(off), d(batch.x), d(batch.y), d(batch.z),
                                  _i32p(morton)) == 0
    # every block is a compact cluster: at 0.09 atoms per A^3 a ball of 64
    # atoms has radius ~5.5 A; the bisection keeps every block within ~2x that,
    # and its largest block is smaller than the Morton order's
    r = radii_of(seg)
    assert r.max() < 12.0, r.max()
    assert r.max() < radii_of(morton[off[0]:off[1]]).max()
    # deterministic (ties by index)
    out2 = np.zeros_like(out)
    lib.gbmc_block_order(batch.n_systems, _i32p(off), d(batch.x), d(batch.y), d(batch.z), _i32p(out2))
    assert np.array_equal(out, out2)
