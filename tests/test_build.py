"""The build entry compiles a clean copy of the tracked sources (no prebuilt library)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not installed")
@pytest.mark.skipif(not os.path.isdir(os.path.join(ROOT, ".git")), reason="not a git checkout")
def test_build_from_clean_tree(tmp_path):
    files = subprocess.run(["git", "ls-files"], cwd=ROOT, capture_output=True, text=True, check=True).stdout.split()
    for f in files:
        src = os.path.join(ROOT, f)
        if not os.path.isfile(src) or f.endswith(".so"):
            continue
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy2(src, dst)
    assert not (tmp_path / "paper_2502_10907_amd" / "libmtf.so").exists()
    code = "import __graft_entry__ as g; g.build(); import paper_2502_10907_amd as m; print(m.LIB_PATH)"
    env = dict(os.environ, PYTHONPATH=str(tmp_path))
    r = subprocess.run([sys.executable, "-c", code], cwd=tmp_path, capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    lib = tmp_path / "paper_2502_10907_amd" / "libmtf.so"
    assert lib.exists() and r.stdout.strip().endswith(str(lib))
