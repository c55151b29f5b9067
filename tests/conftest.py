import json
import os
import shutil
import subprocess
import sys
import tempfile
import time

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FULLSIZE_MODULE = "test_gpu_zfullsize.py"


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle-heavy CPU test (seconds to a minute)")


class OracleWorkers:
    """CPU-only processes computing the full-size oracle references (tests/fullsize_oracle.py)
    while the GPU tests run; `load` waits for one array, printing progress."""

    def __init__(self, config, cases):
        self.config = config
        self.dir = tempfile.mkdtemp(prefix="epr_fullsize_")
        env = dict(os.environ)
        for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            env[v] = "1"
        self.procs = {}
        for case in cases:
            log = open(os.path.join(self.dir, f"{case}.log"), "w")
            self.procs[case] = subprocess.Popen(
                [sys.executable, "-m", "tests.fullsize_oracle", case, self.dir], cwd=ROOT,
                env=env, stdout=log, stderr=subprocess.STDOUT)
        self.t0 = time.time()

    def _say(self, msg):
        capman = self.config.pluginmanager.getplugin("capturemanager")
        if capman is not None:
            with capman.global_and_fixture_disabled():
                print(msg, flush=True)
        else:
            print(msg, flush=True)

    def load(self, case, name, timeout=900):
        path = os.path.join(self.dir, f"{case}.{name}.npy")
        last = 0.0
        while not os.path.exists(path):
            p = self.procs[case]
            if p.poll() is not None and not os.path.exists(path):
                log = open(os.path.join(self.dir, f"{case}.log")).read()[-2000:]
                raise RuntimeError(f"oracle worker {case} exited with {p.returncode}:\n{log}")
            now = time.time() - self.t0
            if now > timeout:
                raise TimeoutError(f"oracle reference {case}.{name} not ready after {now:.0f} s")
            if now - last >= 20.0:
                done = sum(os.path.exists(os.path.join(self.dir, f"{c}.done"))
                           for c in self.procs)
                self._say(f"\n[oracle] waiting for {case}.{name}: {done}/{len(self.procs)} "
                          f"cases done, {now:.0f} s")
                last = now
            time.sleep(1.0)
        return np.load(path)

    def info(self, case):
        path = os.path.join(self.dir, f"{case}.done")
        return json.load(open(path)) if os.path.exists(path) else None

    def close(self):
        for p in self.procs.values():
            if p.poll() is None:
                p.kill()
                p.wait()
        shutil.rmtree(self.dir, ignore_errors=True)


@pytest.hookimpl(trylast=True)
def pytest_collection_modifyitems(session, config, items):
    """Start the oracle workers once the selection (after -m / -k) is known, if it holds a
    full-size test and a device is present."""
    if config.option.collectonly:
        return
    if not any(os.path.basename(str(it.fspath)) == FULLSIZE_MODULE for it in items):
        return
    from tests.helpers import has_gpu
    if not has_gpu():
        return
    from tests import fullsize_oracle as F
    cases = ["nonlocal-poly8-2048", "vjp-poly8-2048", "nonlocal-mono-2048"]
    cases += [f"batch-{i}" for i in sorted(F.batch_indices().values())]
    config._epr_oracle_workers = OracleWorkers(config, cases)


def pytest_unconfigure(config):
    w = getattr(config, "_epr_oracle_workers", None)
    if w is not None:
        w.close()


@pytest.fixture(scope="session")
def oracle_refs(request):
    w = getattr(request.config, "_epr_oracle_workers", None)
    if w is None:
        pytest.skip("full-size oracle references were not started (no device)")
    return w
