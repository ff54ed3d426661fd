"""Plain containers for one calibration problem.

These hold arrays only; no arithmetic of the calibration method lives here.
Arrays may be numpy arrays (host) or torch tensors (host or device).

Layouts (row-major 2x2 Jones matrices, correlation order XX, XY, YX, YY; the
gain vector of one antenna/direction is the row-major vectorisation of its
Jones matrix, paper Section 2.2, eq. gvec / eq. jones):

  data      [n_row][n_chan][4]            complex64 or complex128
  model     [n_row][n_chan][n_dir][4]     same dtype as data
  weight    [n_row][n_chan][n_wcorr]      float32 (c64 data) / float64 (c128)
  flag      [n_row][n_chan]               uint8, nonzero = flagged
  ant1/ant2 [n_row]                       int32 antenna indices p, q
  row_time  [n_row]                       int32 time index, non-decreasing
  chan_freq [n_chan]                      float64, Hz

A chain term (paper eq. joneschain) carries its own solution-interval maps
(paper Section 4.3: data-to-gain mappings instead of broadcasting):

  t_map [n_time] -> [0, n_gt)     f_map [n_chan] -> [0, n_gf)
  d_map [n_dir]  -> [0, n_gdir)
  gains      [n_gt][n_gf][n_ant][n_gdir][4]  complex128  (diag / c2x2 terms)
  params     [n_gt][n_gf][n_ant][n_gdir][2]  float64     (delay: tau_X, tau_Y in s;
                                                        phase: phi_X, phi_Y in rad;
                                                        amplitude: a_X, a_Y;
                                                        delay_offset: [4] phi0_X,
                                                        tau_X, phi0_Y, tau_Y;
                                                        pointing: dl, dm)
  gain_flags [n_gt][n_gf][n_ant][n_gdir]     int8

A pointing term (one parameter pair per antenna whose effect differs by direction)
also carries dir_lm [n_dir][2] (direction cosines of each model direction) and
beam = (fwhm, ref_freq): the full width at half maximum (rad) of its Gaussian
beam at ref_freq (Hz); its d_map is all zeros and n_gdir = 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Any, Optional

TERM_KINDS = ("diag", "c2x2", "delay", "phase", "amplitude", "delay_offset", "pointing")
PARAM_KINDS = ("delay", "phase", "amplitude", "delay_offset", "pointing")


@dataclass
class Vis:
    data: Any
    model: Any
    weight: Any
    flag: Any
    ant1: Any
    ant2: Any
    row_time: Any
    chan_freq: Any
    n_ant: int
    n_time: int

    @property
    def n_row(self) -> int:
        return int(self.data.shape[0])

    @property
    def n_chan(self) -> int:
        return int(self.data.shape[1])

    @property
    def n_dir(self) -> int:
        return int(self.model.shape[2])

    @property
    def n_wcorr(self) -> int:
        return int(self.weight.shape[2])

    def copy(self, **kw) -> "Vis":
        return replace(self, **kw)


@dataclass
class Term:
    kind: str
    t_map: Any
    f_map: Any
    d_map: Any
    n_gt: int
    n_gf: int
    n_gdir: int
    gains: Any = None
    params: Any = None
    gain_flags: Any = None
    direction_dependent: bool = False
    name: str = ""
    dir_lm: Any = None
    beam: Any = None

    def __post_init__(self):
        if self.kind not in TERM_KINDS:
            raise ValueError(f"unknown term kind {self.kind!r}")

    def copy(self, **kw) -> "Term":
        return replace(self, **kw)


@dataclass
class Problem:
    """A visibility set, a Jones chain, and the truth it was generated from."""
    vis: Vis
    chain: list
    truth: list = field(default_factory=list)
    meta: dict = field(default_factory=dict)
