"""The pair-kernel tuner: the automatic configuration is one of its candidates
(storing it changes nothing, bitwise), a tuned size class is never slower
than the automatic configuration in the tuner's own measurement, tuning on
first use fills a persisted table that another context reads back, and
tables of another device kind or malformed ones are refused.  Results of
tuned ensembles match the FP64 oracle (1e-12 FP64, 1e-5 FP32C)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import eval_dev, rod_of, say

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def mrs():
    import paper_2604_12083_amd as m

    return m


def _table(path):
    lines = [ln.split() for ln in open(path).read().splitlines()]
    head = lines[0]
    rows = [[float(x) for x in ln] for ln in lines[1:] if ln and not ln[0].startswith("#")]
    return head, rows


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("nfil,M", [(8, 100), (20, 128), (100, 128)])
def test_automatic_entry_changes_nothing(mrs, prec, nfil, M):
    """The automatic configuration stored as a table entry (chunks = 0)
    keeps its chunking and tail split: same reported configuration and
    bitwise the same velocities as no entry."""
    e = synth.filaments(nfil, M, 4.0 if nfil < 100 else 10.0, 500 + nfil)
    c = mrs.mrs_context_create(0)
    try:
        auto = mrs.mrs_tune_get(c, e.N, prec)
        U0, W0 = eval_dev(mrs, c, e.X, e.f, e.n, e.eps, e.mu, prec)
        mrs.mrs_tune_set(c, e.N, prec, auto["mode"], auto["targets_per_lane"], 0 if auto["mode"] != 1 else 1, 0)
        again = mrs.mrs_tune_get(c, e.N, prec)
        say(f"N={e.N} prec={prec}: automatic {auto}, stored {again}")
        assert again == auto
        U1, W1 = eval_dev(mrs, c, e.X, e.f, e.n, e.eps, e.mu, prec)
        assert np.array_equal(U0, U1) and np.array_equal(W0, W1)
    finally:
        mrs.mrs_context_destroy(c)


def test_first_use_tuning_persists_table(mrs, tmp_path):
    """With tuning on first use, the first evaluation of an ensemble of an
    unseen size class tunes it and writes the table; the tuned entry is at
    least as fast as the automatic one in the tuner's measurement; a second
    context reads the table back and plans the same configuration; the
    tuned ensemble matches the oracle."""
    path = str(tmp_path / "tune.txt")
    e = synth.filaments(24, 128, 6.0, 91)  # 3,072 points: size class 11
    c = mrs.mrs_context_create(0)
    c2 = mrs.mrs_context_create(0)
    try:
        mrs.mrs_tune_on_first_use(c, 1, path)
        for prec in (1, 0):
            h = mrs.mrs_ensemble_create(c, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod_of(mrs, e.rod()))
            try:
                mrs.mrs_ensemble_eval(c, h, prec, False)
                _, _, U, W = mrs.mrs_ensemble_get(c, h)
            finally:
                mrs.mrs_ensemble_destroy(h)
            Uo, Wo = oracle.mrs_eval(e.X, e.f, e.n, e.eps, e.mu)
            eu, ew = oracle.rel_err(U, Uo), oracle.rel_err(W, Wo)
            say(f"first-use tuned prec={prec}: {mrs.mrs_tune_get(c, e.N, prec)} U {eu:.3e} W {ew:.3e}")
            assert eu <= TOL[prec] and ew <= TOL[prec]
        head, rows = _table(path)
        say(f"table: {head} {rows}")
        assert head[0] == "mrs-pair-tuning" and head[1] == "1"
        assert sorted((int(r[0]), int(r[1])) for r in rows) == [(0, 11), (1, 11)]
        for r in rows:
            assert 0 < r[6] <= r[7], r  # tuned median <= automatic median
        mrs.mrs_tune_load(c2, path)
        for prec in (1, 0):
            assert mrs.mrs_tune_get(c2, e.N, prec) == mrs.mrs_tune_get(c, e.N, prec)
        # an entry set by hand is saved with unknown times and read back
        mrs.mrs_tune_set(c2, 40000, 1, 2, 1, 0, 1)
        p2 = str(tmp_path / "tune2.txt")
        mrs.mrs_tune_save(c2, p2)
        c3 = mrs.mrs_context_create(0)
        try:
            mrs.mrs_tune_load(c3, p2)
            assert mrs.mrs_tune_get(c3, 40000, 1) == mrs.mrs_tune_get(c2, 40000, 1)
            assert mrs.mrs_tune_get(c3, e.N, 0) == mrs.mrs_tune_get(c, e.N, 0)
        finally:
            mrs.mrs_context_destroy(c3)
    finally:
        mrs.mrs_context_destroy(c2)
        mrs.mrs_context_destroy(c)


def test_foreign_and_malformed_tables_refused(mrs, tmp_path):
    """A table written for another device kind, a malformed one or a missing
    one (mrs_tune_load) is refused and leaves the table unchanged; a missing
    file is no error for tuning on first use (it is written at once), a path
    that cannot be written is."""
    c = mrs.mrs_context_create(0)
    try:
        own = str(tmp_path / "own.txt")
        mrs.mrs_tune_set(c, 5000, 1, 0, 2, 9, 0)
        mrs.mrs_tune_save(c, own)
        head = open(own).read().splitlines()[0].split()
        before = mrs.mrs_tune_get(c, 20000, 1)
        bad = {
            "arch.txt": f"mrs-pair-tuning 1 gfx000 {head[3]} 0\n1 14 2 1 0 1 -1 -1\n",
            "cus.txt": f"mrs-pair-tuning 1 {head[2]} 7 0\n1 14 2 1 0 1 -1 -1\n",
            "version.txt": f"mrs-pair-tuning 2 {head[2]} {head[3]} 0\n",
            "entry.txt": f"mrs-pair-tuning 1 {head[2]} {head[3]} 0\n1 14 5 1 0 1 -1 -1\n",
            "short.txt": f"mrs-pair-tuning 1 {head[2]} {head[3]} 0\n1 14 2\n",
        }
        for name, text in bad.items():
            p = tmp_path / name
            p.write_text(text)
            with pytest.raises(mrs.MrsError):
                mrs.mrs_tune_load(c, str(p))
            assert mrs.mrs_tune_get(c, 20000, 1) == before, name
        with pytest.raises(mrs.MrsError):
            mrs.mrs_tune_load(c, str(tmp_path / "missing.txt"))
        with pytest.raises(mrs.MrsError):
            mrs.mrs_tune_on_first_use(c, 1, str(tmp_path / "arch.txt"))
        mrs.mrs_tune_on_first_use(c, 1, str(tmp_path / "missing.txt"))
        assert open(tmp_path / "missing.txt").read().startswith("mrs-pair-tuning 1 ")  # written at once
        with pytest.raises(mrs.MrsError):  # a table that cannot be written
            mrs.mrs_tune_on_first_use(c, 1, str(tmp_path / "no_such_dir" / "t.txt"))
        mrs.mrs_tune_on_first_use(c, 0, None)
        with pytest.raises(mrs.MrsError):
            mrs.mrs_tune_on_first_use(c, 21, None)
    finally:
        mrs.mrs_context_destroy(c)


def test_server_and_one_shot_calls_never_tune(mrs, tmp_path):
    """Tuning on first use applies to plans of resident ensembles only: the
    server loop and the one-shot evaluation keep the table as it is."""
    c = mrs.mrs_context_create(0)
    try:
        path = str(tmp_path / "t.txt")
        mrs.mrs_tune_on_first_use(c, 1, path)
        e = synth.filaments(30, 100, 6.0, 93)  # 3,000 points, size class 11
        eval_dev(mrs, c, e.X, e.f, e.n, e.eps, e.mu, 1)
        srv = mrs.mrs_server_start(c, mrs.MRS_FP32C, 1 << 30, 4)
        try:
            t = mrs.mrs_server_submit(srv, 0, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod_of(mrs, e.rod()))
            st, _, _ = mrs.mrs_server_wait(srv, t, e.N, timeout_s=60)
            assert st == mrs.MRS_OK
        finally:
            mrs.mrs_server_stop(srv)
        _, rows = _table(path)
        assert rows == []
        h = mrs.mrs_ensemble_create(c, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod_of(mrs, e.rod()))
        try:
            mrs.mrs_ensemble_eval(c, h, mrs.MRS_FP32C, True)
        finally:
            mrs.mrs_ensemble_destroy(h)
        _, rows = _table(path)
        assert [(int(r[0]), int(r[1])) for r in rows] == [(1, 11)]
    finally:
        mrs.mrs_context_destroy(c)
