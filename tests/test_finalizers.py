"""CPU checks of the binding's finalizers.  A failing test's traceback keeps
its library objects alive until the interpreter exits; their finalizers
then run after the HIP runtime has been torn down, and a library call from
there ended the process with a segmentation fault.  Every handle class
therefore skips its library call while the interpreter finalizes, and
frees its handle through the library otherwise (checked here with a
recording stand-in for the library)."""
import pytest

from paper_2501_18263_amd import heff

CLASSES = [(heff.Context, "heff_destroy"), (heff.Blocks, "heff_blocks_free"), (heff.Davidson, "heff_dav_free"),
           (heff.Batch, "heff_batch_free"), (heff.Su2, "heff_su2_free")]


class _Recorder:
    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        return lambda *a: self.calls.append(name) or 0


@pytest.mark.parametrize("cls,free", CLASSES)
def test_finalizer_skips_library_during_interpreter_exit(monkeypatch, cls, free):
    rec = _Recorder()
    monkeypatch.setattr(heff, "_lib", rec)
    obj = object.__new__(cls)
    obj._h = object()
    obj.__del__(_fin=lambda: True)
    assert rec.calls == [] and obj._h is not None
    obj.__del__(_fin=lambda: False)
    assert rec.calls == [free] and obj._h is None
    obj.__del__(_fin=lambda: False)  # closing twice frees once
    assert rec.calls == [free]
