"""Progress lines of long tests.

A long GPU test prints nothing through pytest's capture until it ends, so its
progress is also appended to gpurun_out/test_progress.log under the repository
root (created if missing), where a watcher of that folder sees it."""
import os
import time

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_T0 = time.perf_counter()


def log(tag: str, msg: str) -> None:
    line = "[%s %.1f s] %s" % (tag, time.perf_counter() - _T0, msg)
    print(line, flush=True)
    try:
        d = os.path.join(_ROOT, "gpurun_out")
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, "test_progress.log"), "a") as f:
            f.write(line + "\n")
    except OSError:
        pass
