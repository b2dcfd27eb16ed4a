"""The benchmark's command line (CPU only): it runs on exactly one GPU and
says so for any other count, before touching a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT,
                          env={**os.environ, **(env or {})})


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run_bench("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def test_world_size_above_one_is_refused():
    r = run_bench("--steps", "1", env={"WORLD_SIZE": "4"})
    assert r.returncode != 0 and "world size 4" in r.stderr


def test_help_lists_the_sections():
    r = run_bench("--help")
    assert r.returncode == 0
    for flag in ("--no-cpu", "--no-batched", "--no-served", "--no-skewed", "--no-lca", "--no-lary",
                 "--no-small", "--no-permutation"):
        assert flag in r.stdout, flag


def test_profile_commands_use_current_flags():
    """Every benchmark command quoted in profiles/ still names flags the
    benchmark accepts, so each summary can be made again as written."""
    import glob
    import re
    help_text = run_bench("--help").stdout
    pdir = os.path.join(ROOT, "profiles")
    seen = 0
    for path in sorted(glob.glob(os.path.join(pdir, "*.md")) + glob.glob(os.path.join(pdir, "*.txt"))):
        for line in open(path, encoding="utf-8"):
            if "bench.py" not in line:
                continue
            tail = line.split("bench.py", 1)[1]
            for flag in re.findall(r"(?<![\w-])--[a-z][a-z0-9-]*", tail):
                assert flag in help_text, (os.path.basename(path), flag)
                seen += 1
    assert seen > 0
