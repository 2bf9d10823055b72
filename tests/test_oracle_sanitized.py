"""The oracle's C loops under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU).  A copy of the oracle library built with -fsanitize=address,undefined
runs, in a child process, Algorithm 1 with uniform and with node2vec walks
(walks, unigram and degree noise tables, training, Psi, the next active set),
the shared-negative step in FP32 and BF16, the FP64 loss and the draws on
small graphs.  Any out-of-bounds access, use after free or undefined
operation in the C code ends the child with an error and fails the test.
The HIP library's host code needs a device for almost every path and is not
covered here."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "felog_oracle.c")

CHILD = r"""
import sys
sys.path.insert(0, sys.argv[2])
import numpy as np
import oracle, synth
oracle._LIB = sys.argv[1]            # the sanitized build, newer than the source
oracle.set_threads(4)
g = synth.csr_from_edges(300, synth.sbm_edges(300, 3, 0.08, 0.01, seed=3))
gw = synth.csr_from_edges(300, synth.sbm_edges(300, 3, 0.08, 0.01, seed=4), weight_seed=5)
common = dict(d=16, r=2, L=12, window=3, K=4, lr0=0.025, lr_end=1e-4, P=256, mu=0.7, k_s=6,
              r_max=2, seed_walk=1, seed_model=2, seed_train=3, seed_psi=4)
tin, tout, st = oracle.run(g, **common)
assert len(st) >= 1 and np.isfinite(tin).all() and np.isfinite(tout).all()
tin, tout, st = oracle.run(gw, walk="node2vec", p=0.5, q=2.0, neg="degree",
                           mode="recompute_all", **common)
assert np.isfinite(tin).all()
walks, capped = oracle.walks_node2vec(gw, np.arange(gw.n, dtype=np.int32), 1, 10, 0.25, 4.0, 7)
assert walks.shape == (gw.n, 10)
cdf = oracle.neg_cdf(oracle.corpus_counts(walks, gw.n))
rng = np.random.default_rng(0)
ctx = rng.integers(0, g.n, 64).astype(np.int32)
ctr = rng.integers(0, g.n, 64).astype(np.int32)
neg = oracle.shared_negatives(0, 0, 64, 9, cdf)
t_in, t_out = oracle.init_tables(g.n, 32, 11)
for bf in (False, True):
    out = oracle.shared_neg_step(t_in, t_out, ctx, ctr, neg, 5, 0.025, bf)
    assert np.isfinite(out[3])
negs = rng.integers(-1, g.n, (64, 4)).astype(np.int32)
loss = oracle.sgns_loss_f64(t_in.astype(np.float64), t_out.astype(np.float64), ctx, ctr, negs)
assert np.isfinite(loss)
xs = rng.integers(0, int(cdf[-1]), 1000, dtype=np.uint64)
ids = oracle.inverse_cdf(cdf, xs)
assert ids.min() >= 0 and ids.max() < gw.n
maps = open("/proc/self/maps").read()
assert "libasan" in maps and sys.argv[1] in maps, "the sanitized build is not the one loaded"
print("sanitized oracle ok", flush=True)
"""


def test_oracle_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not available")
    asan = subprocess.check_output([gcc, "-print-file-name=libasan.so"], text=True).strip()
    if not (os.path.isabs(asan) and os.path.exists(asan)):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call([gcc, "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fopenmp", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
                           "-fno-fast-math", "-o", lib, SRC, "-lm"])
    env = dict(os.environ, LD_PRELOAD=asan, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:exitcode=86",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=87")
    r = subprocess.run([sys.executable, "-c", CHILD, lib, ROOT], env=env, cwd=str(tmp_path),
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, (
        "exit %d\n%s\n%s" % (r.returncode, r.stdout[-2000:], r.stderr[-6000:]))
