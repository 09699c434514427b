"""Host-side checks of bench.py's command-line contract (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env=env, cwd=ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = run_bench("--gpus", "2", "--steps", "3", "--warmup", "1")
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_launched_as_several_ranks_exits_with_a_message():
    env = dict(os.environ, WORLD_SIZE="4", RANK="0", LOCAL_RANK="0")
    r = run_bench("--gpus", "4", env=env)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_profiles_name_the_kernels_bench_reads():
    """The committed counter summary is the one bench.py looks up for the
    dominant kernel's traffic: same workload, digest field present."""
    with open(os.path.join(ROOT, "profiles", "traffic_counters.json")) as fh:
        tc = json.load(fh)
    assert tc["scale"] == 22 and tc["density"] == 0.01
    assert len(tc["source_digest"]) == 16
    for k in ("scan", "scatter", "merge"):
        assert tc["kernels"][k]["fetch_bytes"] > 0 and tc["kernels"][k]["write_bytes"] > 0


def test_profile_commands_run_committed_code_with_known_flags():
    """Every rocprofv3 summary under profiles/ gives the command that made it;
    each must run bench.py from this repository with options it accepts."""
    import glob
    import re
    sys.path.insert(0, ROOT)
    import bench
    parser_src = open(os.path.join(ROOT, "bench.py")).read()
    known = set(re.findall(r'add_argument\("(--[a-z0-9-]+)"', parser_src))
    summaries = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))
    assert summaries
    for path in summaries:
        text = open(path).read()
        cmds = re.findall(r"python3 \$REPO/(\S+)((?: --?[\w-]+(?: [\w.]+)?)*)", text)
        assert cmds, f"{os.path.basename(path)} names no command"
        for script, args in cmds:
            assert script == "bench.py" and os.path.exists(os.path.join(ROOT, script))
            for flag in re.findall(r"(--[a-z0-9-]+)", args):
                assert flag in known, f"{os.path.basename(path)}: bench.py has no {flag}"
    assert callable(bench.kernel_source_digest)
