import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The planted-mistake sweep (test_oracle_mutations.py) runs the oracle pins in
# a child process against a mutated copy of the oracle package placed here.
_ALT_ORACLE = os.environ.get("FE_ORACLE_ROOT")
if _ALT_ORACLE:
    sys.path.insert(0, _ALT_ORACLE)
    import oracle as _oracle
    assert os.path.dirname(os.path.dirname(os.path.abspath(_oracle.__file__))) == os.path.abspath(_ALT_ORACLE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")
