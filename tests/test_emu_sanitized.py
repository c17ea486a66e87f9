"""The library's kernels and C ABI built as host code (tests/emu: a fiber
emulation of wavefronts and workgroups) under AddressSanitizer and
UndefinedBehaviorSanitizer, compared with the oracle. No GPU: this is the
bounds-checked model of every kernel's indexing. Buffers of the emulated
device are exact-size host allocations (distance matrices, swarm states,
batch tables, each workgroup's dynamic LDS), so any access outside one is
reported; waves of a workgroup run in turn between barriers, so a value one
wave stores that another reads without a barrier in between changes the
result (the personal-best race of the move and mutation kernels did)."""
import os
import subprocess
import sys

import pytest

from conftest import ROOT

EMU = os.path.join(ROOT, "tests", "emu")


def _runtime(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()


@pytest.fixture(scope="module")
def emu_lib():
    sys.path.insert(0, EMU)
    import build_emu
    return build_emu.build(verbose=False)


def _run(case, order="fwd", extra=()):
    env = dict(os.environ, LD_PRELOAD=f"{_runtime('libasan.so')}:{_runtime('libubsan.so')}",
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1", EMU_ORDER=order,
               OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, os.path.join(EMU, "run_emu.py"), case, *extra], env=env,
                       capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "EMU RESULT ok" in out, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]


def test_single_swarm_matches_oracle_under_sanitizers(emu_lib):
    _run("quick")


# waves run first to last (wave 0, which holds the lane that stores a block's
# results, always first); EMU_ORDERS="fwd,rev,17" adds reversed and shuffled
# orders
ORDERS = os.environ.get("EMU_ORDERS", "fwd").split(",")


@pytest.mark.parametrize("order", ORDERS)
def test_batch_of_every_class_matches_oracle_under_sanitizers(emu_lib, order):
    """Every edge-exchange class and variant in one batch."""
    _run("batch", order)


def test_every_tuning_matches_oracle_under_sanitizers(emu_lib):
    """Batches and single swarms under six forced tuning tables (threads per
    particle in the move x the exchange's row form)."""
    _run("tuned")


def test_autotune_under_sanitizers(emu_lib):
    """The autotuner's candidates agree, the swarm is left as it was and the
    pick lands in the table."""
    _run("autotune")


def test_batch_orders_under_sanitizers(emu_lib):
    """Index order, longest-first order and XCD groups give the oracle's swarms."""
    _run("orders")


def test_merged_exchange_classes_under_sanitizers(emu_lib):
    """16-bit row classes merged into one launch and launched one after
    another give the oracle's swarms, beside the classes that never merge."""
    _run("merge")
