"""Host-side helpers of bench.py: the kernel-source digest that keys the
committed HBM-traffic summaries, and the cache note of the roofline object."""
import importlib.util
import os
import shutil

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _copy_csrc(tmp_path):
    dst = tmp_path / "paper_2203_01316_amd" / "csrc"
    src = os.path.join(ROOT, "paper_2203_01316_amd", "csrc")
    dst.mkdir(parents=True)
    for name in os.listdir(src):
        if name.endswith((".hip", ".hpp")) or name == "build.py":
            shutil.copy(os.path.join(src, name), dst / name)
    return dst


def test_digest_ignores_comments_but_not_code(bench, tmp_path, monkeypatch):
    dst = _copy_csrc(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.source_digest()
    f = dst / "lbm_impl.hpp"
    text = f.read_text()
    f.write_text("// a new comment line\n" + text.replace("\n", "\n\n", 3) + "\n/* block\n comment */\n")
    assert bench.source_digest() == d0
    f.write_text(text.replace("lds_for_blocks(2)", "lds_for_blocks(3)", 1))
    assert bench.source_digest() != d0


def test_cache_note(bench):
    per_step = 602128944  # 2048^2 coupled FP32 cylinder, bytes moved per step
    assert "partly cache-assisted" in bench.cache_note("aa", per_step)
    assert "cache" not in bench.cache_note("ab", per_step)
    assert "cache" not in bench.cache_note("aa", 4 * per_step)
