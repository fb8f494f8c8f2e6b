"""Progress lines of long GPU tests, printed past pytest's output capture
so that a quiet (-q) run still shows each finished step of a test that
takes minutes."""

CONFIG = None  # set by conftest.pytest_configure


def emit(*args, **kwargs):
    kwargs.setdefault("flush", True)
    capman = CONFIG.pluginmanager.getplugin("capturemanager") if CONFIG is not None else None
    if capman is None:
        print(*args, **kwargs)
        return
    with capman.global_and_fixture_disabled():
        print(*args, **kwargs)
