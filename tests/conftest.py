import pathlib
import sys

ROOT = pathlib.Path(__file__).resolve().parents[1]
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU; runs the HIP path through the C ABI")


def _ensure_built():
    """Build the native libraries once if nothing is built (a fresh checkout)."""
    need = [ROOT / "oracle" / "liboracle.so", ROOT / "gen" / "libeccgen.so",
            ROOT / "paper_1705_02045_amd" / "libecc.so"]
    if not all(p.exists() for p in need):
        import __graft_entry__
        __graft_entry__.build()


_ensure_built()


import pytest  # noqa: E402


@pytest.fixture(autouse=True, scope="module")
def _release_device_memory():
    """After each test module: return the memory its tensors left in torch's
    cache and the library's per-stream scratch, so that a module with large
    images does not leave later modules short of device memory."""
    yield
    import torch
    if not torch.cuda.is_available():
        return
    import paper_1705_02045_amd as ecc
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    ecc.release_workspaces()
