import os
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# launch shapes the library's autotuner persists go to a store of this test
# session, not to the user's
os.environ.setdefault("FVAN_TUNE_FILE", os.path.join(tempfile.mkdtemp(prefix="fvan_tune_"), "tuning.json"))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU oracle checks")
