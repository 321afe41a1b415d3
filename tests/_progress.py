"""Progress lines from inside a test that reach the terminal (or the file a
run is redirected to) at once, while pytest captures the test's own output.
Long GPU tests print one per step so that a slow test is told from a hung one."""
_config = None


def say(msg: str) -> None:
    capman = _config.pluginmanager.getplugin("capturemanager") if _config is not None else None
    if capman is None:
        print(msg, flush=True)
        return
    with capman.global_and_fixture_disabled():
        print(msg, flush=True)
