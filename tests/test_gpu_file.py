"""File-backed streaming: a signal file in, spectra written at the same
relative offsets of an output file, resumable by chunk index."""
import numpy as np
import pytest

import oracle
import paper_1407_6915_amd as fs
import siggen

from gpu_helpers import announce

pytestmark = pytest.mark.gpu


def write_signal(path, sig, samples, header=0):
    x = sig.samples(0, samples)
    with open(path, "wb") as f:
        f.write(b"\x5a" * header)
        f.write(x.tobytes())
    return x


@pytest.mark.parametrize("n,b,chunks", [(4096, 64, 5), (1 << 16, 2, 3)])
def test_file_in_file_out(tmp_path, n, b, chunks):
    announce("file stream n=%d b=%d chunks=%d" % (n, b, chunks))
    sig = siggen.Signal(seed=31, seg_len=n, sigma=1.0, tones=[(9, 0.5, 0.0)])
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    x = write_signal(fin, sig, n * b * chunks, header=4096).reshape(-1, n)
    with fs.Plan(n, b) as p:
        rc, failed, st = p.exec_file(str(fin), str(fout), chunks, in_offset=4096,
                                     io_threads=4)
    assert rc == 0 and failed is None and st["chunks_done"] == chunks
    y = np.fromfile(fout, dtype=np.complex64).reshape(-1, n)
    assert y.shape == x.shape
    err = oracle.rel_l2(y, oracle.fft_recursive(x, n))
    assert np.all(err <= oracle.tolerance(n)), err.max()


def test_file_resume_and_bounds(tmp_path):
    n, b, chunks = 1024, 32, 6
    announce("file stream resume")
    sig = siggen.Signal(seed=32, seg_len=n, sigma=1.0)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    x = write_signal(fin, sig, n * b * chunks).reshape(-1, n)
    chunk = n * b * 8
    with fs.Plan(n, b) as p:
        # chunks 4 and 5 only: written at their own offsets, earlier bytes untouched
        rc, failed, st = p.exec_file(str(fin), str(fout), 2, first_chunk=4)
        assert rc == 0 and st["chunks_done"] == 2
        raw = open(fout, "rb").read()
        assert len(raw) == 6 * chunk and raw[:4 * chunk] == b"\0" * (4 * chunk)
        # then chunks 0..3, completing the file
        rc, failed, st = p.exec_file(str(fin), str(fout), 4, first_chunk=0)
        assert rc == 0
        y = np.fromfile(fout, dtype=np.complex64).reshape(-1, n)
        assert np.all(oracle.rel_l2(y, oracle.fft_recursive(x, n)) <= oracle.tolerance(n))
        # a range past the end of the input file is refused before any work
        with pytest.raises(fs.FFTError) as e:
            p.exec_file(str(fin), str(tmp_path / "o2.bin"), 2, first_chunk=5)
        assert e.value.name == "FFT_ERR_BOUNDS"
        with pytest.raises(fs.FFTError) as e:
            p.exec_file(str(tmp_path / "missing.bin"), str(fout), 1)
        assert e.value.name == "FFT_ERR_INVALID_ARG"
