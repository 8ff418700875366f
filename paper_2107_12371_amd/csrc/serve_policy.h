// Admission policy of the request server: a device-memory budget shared by
// resident matrices and in-flight request buffers, with least-recently-used
// eviction of resident matrices that no in-flight request uses.  Pure C++
// (no HIP), so it is tested on the CPU.
#pragma once

#include <cstdint>
#include <vector>

namespace spmvlib {

class BudgetLRU {
  public:
    enum Verdict : int { ADMIT = 0, WAIT = 1, NEVER = 2 };

    explicit BudgetLRU(uint64_t budget) : budget_(budget) {}

    // Registers a matrix that needs `bytes` of device memory when resident.
    int add_matrix(uint64_t bytes) {
        m_.push_back(Ent{bytes, false, 0, 0});
        return (int)m_.size() - 1;
    }

    // Admits a request on matrix i that also needs `extra` bytes of buffers.
    // ADMIT: the matrix is (or is to be made) resident and the bytes are
    // reserved; `evict` lists the matrices to release first and `upload` is
    // set when matrix i must be uploaded.  WAIT: not enough free memory even
    // after evicting every idle matrix, try again after a completion.
    // NEVER: the request alone exceeds the budget.
    Verdict admit(int i, uint64_t extra, std::vector<int> &evict, bool &upload) {
        evict.clear();
        upload = false;
        Ent &e = m_[i];
        const uint64_t need = extra + (e.resident ? 0 : e.bytes);
        if (e.bytes + extra > budget_) return NEVER;
        uint64_t freeable = 0;
        for (size_t j = 0; j < m_.size(); ++j)
            if ((int)j != i && m_[j].resident && m_[j].pins == 0) freeable += m_[j].bytes;
        if (used_ + need > budget_ + freeable) return WAIT;
        // evict least recently used idle matrices until the request fits
        while (used_ + need > budget_) {
            int victim = -1;
            for (size_t j = 0; j < m_.size(); ++j) {
                if ((int)j == i || !m_[j].resident || m_[j].pins) continue;
                if (victim < 0 || m_[j].last < m_[victim].last) victim = (int)j;
            }
            if (victim < 0) return WAIT;  // unreachable given the check above
            m_[victim].resident = false;
            used_ -= m_[victim].bytes;
            evict.push_back(victim);
            ++evictions_;
        }
        if (!e.resident) {
            e.resident = true;
            used_ += e.bytes;
            upload = true;
            ++uploads_;
        }
        used_ += extra;
        e.pins += 1;
        e.last = ++clock_;
        if (used_ > peak_) peak_ = used_;
        return ADMIT;
    }

    // True when a request on matrix i with `extra` bytes could never fit.
    bool never(int i, uint64_t extra) const { return m_[i].bytes + extra > budget_; }

    // Uploads matrix i ahead of any request if it fits in the free budget
    // without evicting anything; returns whether it was made resident.
    bool preload(int i) {
        Ent &e = m_[i];
        if (e.resident || used_ + e.bytes > budget_) return false;
        e.resident = true;
        used_ += e.bytes;
        e.last = ++clock_;
        ++uploads_;
        if (used_ > peak_) peak_ = used_;
        return true;
    }

    // Holds matrix i against eviction without reserving buffers (an upload
    // in progress); undone by release(i, 0).
    void pin(int i) { m_[i].pins += 1; }

    // A request on matrix i that reserved `extra` bytes has finished.
    void release(int i, uint64_t extra) {
        m_[i].pins -= 1;
        used_ -= extra;
    }

    // Matrix i could not be made resident after an admission that asked for
    // its upload (and whose request has been released): it is not resident.
    void unload(int i) {
        if (!m_[i].resident) return;
        m_[i].resident = false;
        used_ -= m_[i].bytes;
    }

    // Corrects the reservation of a matrix once its true size is known.
    void resize(int i, uint64_t bytes) {
        if (m_[i].resident) used_ = used_ - m_[i].bytes + bytes;
        m_[i].bytes = bytes;
        if (used_ > peak_) peak_ = used_;
    }

    bool resident(int i) const { return m_[i].resident; }
    int pins(int i) const { return m_[i].pins; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    int64_t evictions() const { return evictions_; }
    int64_t uploads() const { return uploads_; }
    uint64_t budget() const { return budget_; }

  private:
    struct Ent {
        uint64_t bytes;
        bool resident;
        int pins;
        uint64_t last;
    };
    uint64_t budget_;
    uint64_t used_ = 0, peak_ = 0, clock_ = 0;
    int64_t evictions_ = 0, uploads_ = 0;
    std::vector<Ent> m_;
};

}  // namespace spmvlib
