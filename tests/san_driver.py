"""Host-side exercise of the C ABI for the sanitizer build (run by
test_host_sanitizers.py in a child process with the sanitizer runtime
preloaded; no device work: every call here returns before any GPU call)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import paper_2005_06191_amd as A  # noqa: E402
import workloads as W  # noqa: E402


def expect_error(fn, *a, **kw):
    try:
        fn(*a, **kw)
    except A.AmyError as e:
        assert len(str(e)) > 10
        return
    raise AssertionError(f"{fn.__name__} accepted an invalid problem")


def main():
    import ctypes
    # the runtime is loaded and the library is the instrumented one
    assert hasattr(ctypes.CDLL(None), "__asan_init"), "AddressSanitizer runtime not loaded"
    assert A.binding.LIB_PATH.endswith("libamytiss_san.so"), A.binding.LIB_PATH
    A.binding.lib()
    print("version", A.version())
    beta = dict(noise="beta", noise_a=(-0.05,) * 5, noise_b=(0.05,) * 5, noise_alpha=(2.0,) * 5,
                noise_beta=(2.0,) * 5)
    probs = [W.unicycle3d(), W.room5d(), W.vehicle7d(), W.linear2d(mode="stored"), W.linear2d(mode="otf"),
             W.robot2d(), W.traffic5d(q=0.74), W.room5d().with_(**beta), W.room5d().with_(window="intersect"),
             W.linear2d().with_(multiplicative=True), W.room5d(precision="fp64"),
             W.unicycle3d().with_(noise="uniform", noise_a=(-0.01,) * 3, noise_b=(0.01,) * 3),
             W.linear2d().with_(noise="exponential", noise_a=(25.0, 40.0), cutoff=1e-2)]
    for p in probs:
        for variant in ("auto", "lanes", "fixed", "factored", "group16", "group64", "inputs"):
            try:
                q = A.query(p, variant=variant)
                assert q["W"] > 0 and q["rows"] > 0
            except A.AmyError as e:
                assert e.status in (A.binding.E_UNSUPPORTED, A.binding.E_INVALID, A.binding.E_NOMEM), e
        expect_error(A.query, p.with_(mode="stored"), budget=1 << 10)
    bad = [dict(var=(0.0, 0.01)), dict(h=(-0.04, 0.04)), dict(count=(0, 50)), dict(horizon=-1),
           dict(cutoff=-1e-3), dict(cutoff=10.0), dict(params=(1.0, 2.0)), dict(noise="beta"),
           dict(noise="uniform", noise_a=(0.1, 0.1), noise_b=(0.0, 0.2)), dict(count=(50000, 50000)),
           dict(w_lo=(0.0,) * 4, w_hi=(1.0,) * 4, w_count=(2,) * 4)]
    for kw in bad:
        expect_error(A.query, W.linear2d().with_(**kw))
    # a disturbance on a family that takes none
    expect_error(A.query, W.room5d().with_(w_lo=(0.0,), w_hi=(1.0,), w_count=(2,)))
    expect_error(A.grid_from_quantization, [0.0], [1.0], [0.0])
    expect_error(A.grid_from_quantization, [1.0], [0.0], [0.1])
    print(A.grid_from_quantization([-10.0, -10.0], [10.0, 10.0], [0.5, 0.5]))
    print(A.inputs_from_quantization([-1.0, -1.0], [1.0, 1.0], [0.2, 0.2]))
    n = A.batch_query([W.linear2d(cells=c, mode="otf") for c in (17, 33, 65)])
    assert n > 0
    # the tuning cache: save, clear, load, and a malformed file
    path = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"amy_san_tune_{os.getpid()}.txt")
    A.tune_save(path)
    A.tune_clear()
    A.tune_load(path)
    with open(path, "w") as fh:
        fh.write("not a cache\n1 2 3\n")
    try:
        A.tune_load(path)
    except A.AmyError:
        pass
    os.remove(path)
    print("san driver ok", A.tune_entries())


if __name__ == "__main__":
    main()
