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


def test_committed_profiles_match_the_kernel_source():
    """The committed HBM-traffic summary of the full-force launch was taken on the current
    kernel source (bench.py reports its figure only then), and every committed summary names
    the command that produced it."""
    import json
    from paper_astro_ph_0702058_amd.profiling import kernel_source_hash
    prof = os.path.join(ROOT, "profiles")
    t = json.load(open(os.path.join(prof, "force_full_fp32_plummer_n1048576_traffic.json")))
    assert t["kernel_source_sha256_16"] == kernel_source_hash()
    assert t["variant"] == {"ipl": 1, "unroll": 2, "target": 65536, "kmax": 64}
    assert set(t["commands"]) == {"FETCH_SIZE", "WRITE_SIZE"}
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
