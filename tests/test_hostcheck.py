"""CPU host check of the library's host code (no GPU).

csrc/heff_host.hip is compiled with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer against a host-only HIP runtime
(tests/hostcheck/): device memory is host memory whose allocations are
tracked, and every kernel launcher is replaced by a checker that verifies,
for each work item, tile and task the launch would run, that every operand
block, output block and table entry lies inside one live allocation, that
identity operands have matching dimensions and that blocks fit their kernel
variant (the shapes the kernels and their grids assume).  The driver builds
the blocks and task tables of each problem through the C ABI, runs single
products in all precisions and the diagonal, and a batch of all problems
with plain launches and with captured graphs replayed over the autotuner's
grid sweep."""
import os
import struct
import subprocess

import numpy as np
import pytest

from paper_2501_18263_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HC = os.path.join(ROOT, "tests", "hostcheck")
SRC = [os.path.join(ROOT, "paper_2501_18263_amd", "csrc", "heff_host.hip"),
       os.path.join(ROOT, "paper_2501_18263_amd", "csrc", "heff_su2.hip"),
       os.path.join(HC, "hostcheck_runtime.cpp"), os.path.join(HC, "hostcheck_main.cpp")]


def build_hostcheck(out_dir):
    """g++ build of the host code against the host-only runtime, with the
    address and undefined-behaviour sanitizers; returns the executable."""
    exe = os.path.join(out_dir, "hostcheck")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-I" + HC, "-I" + os.path.join(ROOT, "paper_2501_18263_amd", "csrc"), "-I" + os.path.join(ROOT, "include"),
           "-x", "c++", SRC[0], SRC[1], "-x", "none", SRC[2], SRC[3], "-o", exe, "-lpthread"]
    subprocess.check_call(cmd)
    return exe


def write_problems(path, problems):
    """Problem file of the driver (format in hostcheck_main.cpp)."""
    with open(path, "wb") as f:
        f.write(b"HEFFPRB1")
        f.write(struct.pack("<i", len(problems)))
        for p in problems:
            f.write(struct.pack("<iii", p.n_orb, p.n_up, p.n_dn))
            f.write(np.ascontiguousarray(p.h, dtype="<f8").tobytes())
            f.write(np.ascontiguousarray(p.V, dtype="<f8").tobytes())
            for tabs in (p.left, p.right):
                f.write(struct.pack("<i", len(tabs)))
                for t in tabs:
                    f.write(struct.pack("<i", len(t)))
                    for col in (0, 1):
                        f.write(np.array([q[col] for q in t], dtype="<i4").tobytes())
                    f.write(np.array(list(t.values()), dtype="<i4").tobytes())
            for tabs, isos in ((p.left, p.iso_left), (p.right, p.iso_right)):
                f.write(struct.pack("<i", len(isos)))
                for i, blocks in enumerate(isos):
                    a = np.ascontiguousarray(synth.iso_flat(tabs[i], tabs[i + 1], blocks), dtype="<f8")
                    f.write(struct.pack("<q", a.size))
                    f.write(a.tobytes())


def run_hostcheck(exe, path, single=True, timeout=600):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    args = [exe, path] + ([] if single else ["--no-single"])
    r = subprocess.run(args, capture_output=True, text=True, timeout=timeout, env=env)
    return r


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if subprocess.run(["g++", "--version"], capture_output=True).returncode != 0:
        pytest.skip("no g++")
    return build_hostcheck(str(tmp_path_factory.mktemp("hostcheck")))


def _summary(r):
    import json
    assert r.returncode == 0, (r.returncode, r.stdout[-3000:], r.stderr[-6000:])
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_hostcheck_small_problems(exe, tmp_path):
    # small problems of every kind the library builds: even and odd N (odd N
    # has S_z = +1/2), truncated and complete blocks, one work-group rows
    probs = [synth.make_problem(6, 16, 3), synth.make_problem(7, 32, 2), synth.make_problem(8, 64, 1),
             synth.make_problem(9, 48, 4), synth.make_problem(10, 48, 7, beta=1.0)]
    path = str(tmp_path / "small.bin")
    write_problems(path, probs)
    s = _summary(run_hostcheck(exe, path))
    assert s["violations"] == 0 and s["leaked_bytes"] == 0 and s["leaked_allocations"] == 0
    assert s["work_items_checked"] > 0 and s["tasks_checked"] > 0


def test_hostcheck_batch_sample(exe, tmp_path):
    # problems of the batched workload's list (N uniform in 12..28, D in
    # {128, 256, 512, 1024}; here the first six with N <= 20 and D <= 256,
    # to keep the sanitized run short; all 64 pass as well), batch built and
    # replayed
    specs = [s for s in synth.batch_specs(64) if s[0] <= 20 and s[1] <= 256][:6]
    probs = [synth.make_problem(n, d, sd) for n, d, sd in specs]
    path = str(tmp_path / "batch.bin")
    write_problems(path, probs)
    s = _summary(run_hostcheck(exe, path, single=False))
    assert s["violations"] == 0 and s["leaked_bytes"] == 0 and s["leaked_allocations"] == 0


def write_su2_problems(path, problems):
    """SU(2) problem file of the driver (format in hostcheck_main.cpp)."""
    from paper_2501_18263_amd import synth_su2
    with open(path, "wb") as f:
        f.write(b"HEFFSU21")
        f.write(struct.pack("<i", len(problems)))
        for p in problems:
            for blk in (p.L, p.R):
                sec = np.array(blk.sectors, dtype="<i4").reshape(-1, 3)
                f.write(struct.pack("<i", len(sec)))
                for j in range(3):
                    f.write(np.ascontiguousarray(sec[:, j]).tobytes())
                f.write(struct.pack("<i", len(blk.ops)))
                f.write(np.array([op[0] for op in blk.ops], dtype="<i4").tobytes())
                f.write(np.array([op[1] for op in blk.ops], dtype="<i4").tobytes())
                bop, bout, bin_, boff, data = synth_su2.op_arrays(blk)
                f.write(struct.pack("<q", len(bop)))
                for a in (bop, bout, bin_):
                    f.write(a.astype("<i4").tobytes())
                f.write(boff.astype("<i8").tobytes())
                f.write(struct.pack("<q", data.size))
                f.write(data.astype("<f8").tobytes())
            f.write(struct.pack("<i", len(p.terms)))
            for j in range(5):
                f.write(np.array([t[j] for t in p.terms], dtype="<i4").tobytes())
            f.write(np.array([t[5] for t in p.terms], dtype="<f8").tobytes())
            f.write(struct.pack("<ii", p.n_tot, p.ts_tot))


def test_hostcheck_su2(exe, tmp_path):
    # the SU(2) product's validation, layout and task table on small and
    # medium problems (every spin total up to 3/2, dimensions up to 70 so
    # that output blocks span two 64-row work items), launched in every
    # precision through the checkers
    from paper_2501_18263_amd import synth_su2 as S
    probs = []
    for seed, (n_tot, ts) in enumerate([(4, 0), (4, 2), (3, 1), (5, 3)]):
        p = S.small_problem(seed + 1)
        p.n_tot, p.ts_tot = n_tot, ts
        probs.append(p)
    rng = np.random.default_rng(9)
    Ls = S.sectors(rng, range(2, 7), 5, 70, 20)
    Rs = S.sectors(rng, range(2, 7), 5, 70, 20)
    probs.append(S.make_problem(9, Ls, Rs, 16, 16, 120, 9, 1))
    # right sectors up to 200 wide next to narrow ones: tasks with a middle
    # dimension above 128 into outputs at most 128 wide
    rng = np.random.default_rng(10)
    Ls = S.sectors(rng, range(2, 5), 3, 24, 4)
    Rs = [(2, 0, 200), (2, 2, 40), (3, 1, 150), (3, 3, 20), (4, 0, 90), (4, 2, 130)]
    probs.append(S.make_problem(11, Ls, Rs, 12, 12, 60, 7, 1))
    path = str(tmp_path / "su2.bin")
    write_su2_problems(path, probs)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, "--su2", path], capture_output=True, text=True, timeout=600, env=env)
    s = _summary(r)
    assert s["violations"] == 0 and s["leaked_bytes"] == 0 and s["leaked_allocations"] == 0
    assert s["tasks"] > 0 and s["work_items_checked"] > 0 and s["tasks_checked"] > 0
