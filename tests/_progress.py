"""Progress lines of long GPU tests, written to the terminal as they happen
(pytest captures a test's own output until the test ends)."""
import contextlib
import sys

CONFIG = None


def say(*parts):
    msg = " ".join(str(p) for p in parts)
    pm = CONFIG.pluginmanager if CONFIG is not None else None
    tr = pm.getplugin("terminalreporter") if pm is not None else None
    if tr is None:
        print(msg, flush=True)
        return
    capman = pm.getplugin("capturemanager")
    ctx = capman.global_and_fixture_disabled() if capman is not None else contextlib.nullcontext()
    with ctx:
        tr.ensure_newline()
        tr.write(msg + "\n", flush=True)
        sys.stdout.flush()
