// Event-pair timing of library kernel launches (see shtn_profile_* in shtn.h).
#pragma once

namespace shtn {

enum ProfKind { PK_PRESCALE = 0, PK_LEG_SYNTH = 1, PK_LEG_ANALYS = 2, PK_C2R = 3, PK_R2C = 4 };
constexpr int kProfKinds = 5;

// While set (per thread), ProfScope records nothing: used around stream
// capture, where event records would become graph nodes.
void prof_set_capturing(bool on);

// Records a start event on construction and a stop event on destruction when
// profiling is enabled; otherwise does nothing.
class ProfScope {
public:
    ProfScope(int kind, void* stream);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

private:
    int kind_;
    void* stream_;
    void* ev_ = nullptr;
};

}  // namespace shtn
