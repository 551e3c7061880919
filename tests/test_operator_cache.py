"""The on-disk operator cache (host only): the FP64 operator precomputation
of Sec. II stored per (order, boundary, cuts, operator sources) and loaded
by later processes.  A loaded set must be the built one bit for bit (equal
digests); damaged, truncated or foreign files are rebuilt; concurrent
writers leave one whole file; an unusable directory only costs the rebuild."""
import multiprocessing as mp
import os

import pytest

from paper_2010_15155_amd import StkfmmError, prepare_operators


def _files(d, pattern="*.bin"):
    return sorted(d.glob(pattern))


def test_store_then_load(tmp_path):
    built = prepare_operators(6, "open", 1e-7, 2e-7)                 # no cache
    first = prepare_operators(6, "open", 1e-7, 2e-7, cache_dir=str(tmp_path))
    second = prepare_operators(6, "open", 1e-7, 2e-7, cache_dir=str(tmp_path))
    assert first == (False, built[1])
    assert second == (True, built[1])
    assert len(_files(tmp_path, "ops_p6_open_*.bin")) == 1
    assert not _files(tmp_path, "*.tmp.*")


def test_parameters_select_files(tmp_path):
    d = str(tmp_path)
    sets = [(5, "open", 1e-7, 0.0), (5, "open", 1e-7, 2e-7), (5, "open", 1e-9, 2e-7), (4, "open", 1e-7, 0.0),
            (4, "wall", 1e-7, 0.0)]
    digests = []
    for s in sets:
        loaded, dg = prepare_operators(*s, cache_dir=d)
        digests.append(dg)
    # the wall's summations use the open operator set: same file, same digest
    assert len(_files(tmp_path)) == 4
    assert digests[3] == digests[4]
    assert len(set(digests[:4])) == 4
    for s, dg in zip(sets, digests):
        assert prepare_operators(*s, cache_dir=d) == (True, dg)


def test_damaged_files_are_rebuilt(tmp_path):
    d = str(tmp_path)
    _, dg = prepare_operators(5, "open", 1e-7, 2e-7, cache_dir=d)
    (f,) = _files(tmp_path)
    good = f.read_bytes()
    flipped = bytearray(good)
    flipped[len(good) // 2] ^= 0x40
    for bad in (bytes(flipped), good[: len(good) // 2], good + b"\0" * 8, good[:12], b""):
        f.write_bytes(bad)
        assert prepare_operators(5, "open", 1e-7, 2e-7, cache_dir=d) == (False, dg)
        assert f.read_bytes() == good                  # rewritten whole
        assert prepare_operators(5, "open", 1e-7, 2e-7, cache_dir=d) == (True, dg)


def test_unusable_directory_still_builds(tmp_path):
    blocker = tmp_path / "not_a_dir"
    blocker.write_bytes(b"x")
    _, dg = prepare_operators(4, "open", 1e-7, 0.0)
    assert prepare_operators(4, "open", 1e-7, 0.0, cache_dir=str(blocker / "cache")) == (False, dg)
    assert prepare_operators(4, "open", 1e-7, 0.0, cache_dir="") == (False, dg)


def _prepare(d):
    return prepare_operators(6, "open", 1e-7, 2e-7, cache_dir=d)


def test_concurrent_writers_leave_one_whole_file(tmp_path):
    d = str(tmp_path / "nested" / "cache")
    with mp.get_context("spawn").Pool(4) as pool:
        res = pool.map(_prepare, [d] * 4)
    assert len({dg for _, dg in res}) == 1
    files = _files(tmp_path / "nested" / "cache")
    assert len(files) == 1 and not _files(tmp_path / "nested" / "cache", "*.tmp.*")
    assert _prepare(d) == (True, res[0][1])


@pytest.mark.slow
def test_periodic_far_images_are_cached(tmp_path):
    # the doubly periodic plan's far-image fit (Ewald sums at order 10) is the
    # costliest part to build; PXY adds it to the open set
    d = str(tmp_path)
    first = prepare_operators(4, "PXY", 1e-7, 0.0, cache_dir=d)
    assert first[0] is False
    assert len(_files(tmp_path, "stkfar_p10_pxy_*.bin")) == 1
    assert prepare_operators(4, "PXY", 1e-7, 0.0, cache_dir=d) == (True, first[1])


@pytest.mark.parametrize("args", [(1, "open", 1e-7, 0.0), (17, "open", 1e-7, 0.0), (6, "PX", 1e-7, 0.0),
                                  (6, "open", 0.0, 0.0), (6, "open", 1e-7, 1.0), (6, "open", 1e-7, -1e-3)])
def test_rejects_bad_arguments(args, tmp_path):
    with pytest.raises(StkfmmError) as ei:
        prepare_operators(*args, cache_dir=str(tmp_path))
    assert ei.value.status == "E_ARG"
    assert not _files(tmp_path)
