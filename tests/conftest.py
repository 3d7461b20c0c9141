import os
import sys

# the oracle's C core runs OpenMP loops between numpy's (OpenBLAS) dense
# eigen-solves: idle OpenMP threads that spin instead of sleeping slow those
# solves down many times over on a shared CPU
os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")
