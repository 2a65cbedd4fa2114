"""Host-side checks that need no GPU: the C-ABI library loads, exports every entry point the
header declares, and the product package never reaches the oracle."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")
PKG = os.path.join(ROOT, "paper_astro_ph_0702058_amd")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nb_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_astro_ph_0702058_amd import nbody
    if not os.path.exists(nbody.LIB_PATH):
        from paper_astro_ph_0702058_amd import build
        build.build()
    return nbody.load_library()


def test_exports_every_declared_symbol(lib):
    from paper_astro_ph_0702058_amd import nbody
    declared = _declared()
    assert len(declared) >= 19
    out = subprocess.run(["nm", "-D", "--defined-only", nbody.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (nb_\w+)", out))
    missing = [d for d in declared if d not in exported]
    assert not missing, missing
    assert sorted(nbody.EXPORTS) == declared


def test_version_and_argument_errors(lib):
    import ctypes
    from paper_astro_ph_0702058_amd import nbody
    assert b"gfx950" in lib.nb_version()
    # argument checks happen before any device work
    assert lib.nb_create(None, 10, 0.1, 3, 26, 0) == nbody.NB_EINVAL
    h = ctypes.c_void_p()
    assert lib.nb_create(ctypes.byref(h), 0, 0.1, 3, 26, 0) == nbody.NB_EINVAL
    assert lib.nb_create(ctypes.byref(h), 10, -1.0, 3, 26, 0) == nbody.NB_EINVAL
    assert lib.nb_create(ctypes.byref(h), 10, 0.1, 5, 4, 0) == nbody.NB_EINVAL
    assert lib.nb_create(ctypes.byref(h), 10, 0.1, 3, 26, 7) == nbody.NB_EINVAL
    assert lib.nb_destroy(None) == nbody.NB_OK
    assert lib.nb_init(None, 0.01) == nbody.NB_EINVAL
    assert lib.nb_force(None, None, None, 1, None, None, None) == nbody.NB_EINVAL


def test_library_is_gfx950_code_object():
    from paper_astro_ph_0702058_amd import nbody
    data = open(nbody.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_product_never_imports_oracle():
    """The product path has no CPU fallback: nothing under the package names the oracle."""
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, re.M), f
                assert "nbody_oracle" not in text, f


def test_missing_library_fails_loudly(tmp_path):
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_astro_ph_0702058_amd import nbody\n"
            "try:\n    nbody.load_library(%r)\nexcept RuntimeError as e:\n    print('raised', e)\n"
            % (ROOT, str(tmp_path / "nope.so")))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert "raised" in r.stdout


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: any --gpus other than 1 exits with status 2 and a message,
    before touching a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_committed_traffic_is_reported_only_for_its_kernel_source():
    """The committed HBM-traffic summary of the full-force launch names its kernel source hash,
    launch variant and the two counter commands; bench.py reports its figure only while the
    kernel source, the workload and the launch variant are the ones the counters were taken
    with, and null otherwise.  Every committed summary names the command that produced it."""
    import json
    import types
    sys.path.insert(0, ROOT)
    import bench
    from paper_astro_ph_0702058_amd.profiling import kernel_source_hash
    prof = os.path.join(ROOT, "profiles")
    t = json.load(open(os.path.join(prof, "force_full_fp32_plummer_n1048576_traffic.json")))
    assert set(t["commands"]) == {"FETCH_SIZE", "WRITE_SIZE"}
    assert t["hbm_bytes_per_launch"] > 0
    args = types.SimpleNamespace(eps=t["eps"])
    got = bench.committed_traffic(t["kernel"], t["n"], args, t["variant"])
    if t["kernel_source_sha256_16"] == kernel_source_hash():
        assert got == t["hbm_bytes_per_launch"]
    else:
        assert got is None
    assert bench.committed_traffic(t["kernel"], t["n"] // 2, args, t["variant"]) is None
    other = dict(t["variant"], unroll=t["variant"]["unroll"] + 1)
    assert bench.committed_traffic(t["kernel"], t["n"], args, other) is None
    for name in os.listdir(prof):
        if name.endswith(".txt"):
            assert "# command: " in open(os.path.join(prof, name)).read(), name


def test_binding_rejects_host_tensors_and_wrong_index_types():
    """nb_force arguments are checked on the host before any launch: host tensors, another
    element type (an int64 index list would be read as int32 pairs on the device), wrong shapes
    and out-of-range indices raise; the checks need no GPU (they stop at the first problem)."""
    import torch
    from paper_astro_ph_0702058_amd import nbody
    n = 8
    acc = torch.zeros((3, n), dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU tensor"):
        nbody.check_force_args(n, acc, acc, acc[0], None, None, n)
    with pytest.raises(TypeError, match="dtype"):
        nbody._device_tensor(torch.zeros(3, dtype=torch.int64), "i_idx", torch.int32)
    with pytest.raises(ValueError, match="n_i_max"):
        nbody.check_force_args(n, acc, acc, acc[0], None, None, n + 1)
    with pytest.raises(TypeError, match="torch tensor"):
        nbody.check_force_args(n, np.zeros((3, n)), acc, acc[0], None, None, n)


def test_scratch_bytes(lib):
    """The workspace size of a context (no device needed): 0 for invalid arguments; at least
    the fixed per-particle buffers (j-stream 64 B, block outputs 56 B, block list 4 B, criterion
    16 B, energy 64 B, adjoint 96 B: 300 B per particle) and at most those plus 64 j-ranges of
    partial sums (56 B per particle each) and small records; growing with n.  The ensemble's
    likewise: at least its block list and criterion plus one partial plane set per cluster."""
    import ctypes
    lib.nb_scratch_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.nb_scratch_bytes.restype = ctypes.c_size_t
    assert lib.nb_scratch_bytes(0, 0) == 0 and lib.nb_scratch_bytes(10, 9) == 0
    prev = 0
    for n in (1, 1000, 65536, 1 << 20):
        for prec in range(5):
            b = lib.nb_scratch_bytes(n, prec)
            assert 300 * n <= b <= 300 * n + 64 * 56 * n + (1 << 20), (n, prec, b)
        b = lib.nb_scratch_bytes(n, 0)
        assert b > prev
        prev = b
    lib.nb_ens_scratch_bytes.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32]
    lib.nb_ens_scratch_bytes.restype = ctypes.c_size_t
    off = np.array([0, 100, 300, 4396], np.int32)
    b = lib.nb_ens_scratch_bytes(3, off.ctypes.data_as(ctypes.c_void_p), 0)
    tiles = [(100 + 255) // 256, (200 + 255) // 256, (4096 + 255) // 256]
    planes = 8 * 7 * (tiles[0] * 100 + tiles[1] * 200 + tiles[2] * 4096)
    assert 20 * 4396 + planes <= b <= 20 * 4396 + planes + (1 << 16), b
    bad = np.array([0, 100, 100, 200], np.int32)
    assert lib.nb_ens_scratch_bytes(3, bad.ctypes.data_as(ctypes.c_void_p), 0) == 0
    assert lib.nb_ens_scratch_bytes(3, off.ctypes.data_as(ctypes.c_void_p), 3) == 0


def test_bench_oracle_reference_cache(tmp_path):
    """The benchmark's cache of oracle reference rows: a stored reference comes back bitwise for
    the same input and rows, and any change of input, softening or rows misses."""
    import bench
    rng = np.random.default_rng(3)
    x, v = rng.normal(size=(50, 3)), rng.normal(size=(50, 3))
    m = np.full(50, 1 / 50)
    idx = np.arange(0, 50, 7, dtype=np.int64)
    ref = (rng.normal(size=(idx.size, 3)), rng.normal(size=(idx.size, 3)), rng.normal(size=idx.size))
    d = str(tmp_path)
    assert bench.load_oracle_reference(d, x, v, m, 0.01, idx) is None
    bench.save_oracle_reference(d, x, v, m, 0.01, idx, ref)
    got = bench.load_oracle_reference(d, x, v, m, 0.01, idx)
    assert all(np.array_equal(a, b) for a, b in zip(got, ref))
    x2 = x.copy(); x2[3, 1] += 1e-12
    assert bench.load_oracle_reference(d, x2, v, m, 0.01, idx) is None
    assert bench.load_oracle_reference(d, x, v, m, 0.02, idx) is None
    assert bench.load_oracle_reference(d, x, v, m, 0.01, idx[1:]) is None
    assert bench.load_oracle_reference("", x, v, m, 0.01, idx) is None
